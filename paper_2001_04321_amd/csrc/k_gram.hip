// Factor Grams A^T A and their Hadamard product (paper Appendix A gradient: the r x r
// matrix (B^(n))^T B^(n) equals the Hadamard product of the other factors' Grams).
//
// gram_partials: block (c, f) stages one row chunk of factor f in LDS and writes its
// float64 partial Gram (chunk_gram). hadamard: sums each factor's partials in chunk order
// and multiplies them entrywise; it can also reset the inner solver's wait slots for the
// next A-HALS launch. All reductions have a fixed order, so results are deterministic.
#include "gram_chunk.h"
#include "ntf_internal.h"

namespace ntf {
namespace {

__global__ __launch_bounds__(256) void gram_partials_kernel(GramJob job, int r) {
  extern __shared__ float s_rows[];  // chunk x r
  const int f = blockIdx.y;
  if (f >= job.nfac) return;
  const int64_t rows = job.rows[f];
  const int chunk = gram_chunk_rows(r, rows);
  const int64_t c = blockIdx.x;
  const int64_t r0 = c * chunk;
  if (r0 >= rows) return;
  const int nrows = int(std::min<int64_t>(chunk, rows - r0));
  const float* A = job.A[f] + r0 * r;
  for (int e = threadIdx.x; e < nrows * r; e += blockDim.x) s_rows[e] = A[e];
  __syncthreads();
  chunk_gram(s_rows, nrows, r, job.out[f] + c * int64_t(r) * r);
}

__global__ __launch_bounds__(256) void hadamard_kernel(HadamardJob job, int r, float* G32,
                                                       double* G64, double* slots,
                                                       int64_t nslots) {
  hadamard_work(job, r, G32, G64, slots, nslots, blockIdx.x, gridDim.x);
}

}  // namespace

int64_t gram_chunks(int64_t rows, int r) { return ceil_div(rows, gram_chunk_rows(r, rows)); }

hipError_t launch_gram_partials(const GramJob& job, int r, hipStream_t s) {
  int64_t maxc = 1;
  int maxrows = 1;
  for (int f = 0; f < job.nfac; ++f) {
    maxc = std::max(maxc, gram_chunks(job.rows[f], r));
    maxrows = std::max(maxrows, gram_chunk_rows(r, job.rows[f]));
  }
  const size_t lds = size_t(maxrows) * r * sizeof(float);
  hipLaunchKernelGGL(gram_partials_kernel, dim3(unsigned(maxc), unsigned(job.nfac)), dim3(256),
                     lds, s, job, r);
  return hipGetLastError();
}

hipError_t launch_hadamard(const HadamardJob& job, int r, float* G32, double* G64,
                           double* slots, int64_t nslots, hipStream_t s) {
  const int64_t work = std::max<int64_t>(4 * int64_t(r) * r, nslots);  // four threads per entry
  const int blocks = int(std::max<int64_t>(1, std::min<int64_t>(ceil_div(work, 256), 1024)));
  hipLaunchKernelGGL(hadamard_kernel, dim3(blocks), dim3(256), 0, s, job, r, G32, G64, slots,
                     nslots);
  return hipGetLastError();
}

}  // namespace ntf
