// Factor Grams A^T A and their Hadamard product (paper Appendix A gradient: the r x r
// matrix (B^(n))^T B^(n) equals the Hadamard product of the other factors' Grams).
//
// gram_partials: block (c, f) stages kGramChunk rows of factor f in LDS and writes the
// float64 partial Gram of those rows (products of float32 values are exact in float64).
// hadamard: sums each factor's partials in chunk order and multiplies them entrywise.
// Both reductions have a fixed order, so results are deterministic.
#include "ntf_internal.h"

namespace ntf {
namespace {

constexpr int kEntriesPerPass = 16;  // Gram entries accumulated per thread per pass

__global__ __launch_bounds__(256) void gram_partials_kernel(GramJob job, int r) {
  extern __shared__ float s_rows[];  // kGramChunk x r
  const int f = blockIdx.y;
  if (f >= job.nfac) return;
  const int64_t rows = job.rows[f];
  const int64_t c = blockIdx.x;
  const int64_t r0 = c * kGramChunk;
  if (r0 >= rows) return;
  const int nrows = int(std::min<int64_t>(kGramChunk, rows - r0));
  const float* A = job.A[f] + r0 * r;
  for (int e = threadIdx.x; e < nrows * r; e += blockDim.x) s_rows[e] = A[e];
  __syncthreads();
  double* out = job.out[f] + c * int64_t(r) * r;
  const int rr = r * r;
  for (int base = 0; base < rr; base += 256 * kEntriesPerPass) {
    double acc[kEntriesPerPass];
    int pp[kEntriesPerPass], qq[kEntriesPerPass];
#pragma unroll
    for (int t = 0; t < kEntriesPerPass; ++t) {
      const int e = base + t * 256 + threadIdx.x;
      acc[t] = 0.0;
      pp[t] = e < rr ? e / r : 0;
      qq[t] = e < rr ? e % r : 0;
    }
    for (int i = 0; i < nrows; ++i) {
      const float* row = s_rows + i * r;
#pragma unroll
      for (int t = 0; t < kEntriesPerPass; ++t)
        acc[t] += double(row[pp[t]]) * double(row[qq[t]]);
    }
#pragma unroll
    for (int t = 0; t < kEntriesPerPass; ++t) {
      const int e = base + t * 256 + threadIdx.x;
      if (e < rr) out[e] = acc[t];
    }
  }
}

__global__ __launch_bounds__(256) void hadamard_kernel(HadamardJob job, int r, float* G32,
                                                       double* G64) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int rr = r * r;
  if (e >= rr) return;
  double g = 1.0;
  for (int f = 0; f < job.nfac; ++f) {
    double s = 0.0;
    const double* part = job.part[f];
    for (int64_t c = 0; c < job.nchunks[f]; ++c) s += part[c * rr + e];
    g *= s;
  }
  if (G32) G32[e] = float(g);
  if (G64) G64[e] = g;
}

}  // namespace

int64_t gram_chunks(int64_t rows) { return ceil_div(rows, kGramChunk); }

hipError_t launch_gram_partials(const GramJob& job, int r, hipStream_t s) {
  int64_t maxc = 1;
  for (int f = 0; f < job.nfac; ++f) maxc = std::max(maxc, gram_chunks(job.rows[f]));
  const size_t lds = size_t(kGramChunk) * r * sizeof(float);
  hipLaunchKernelGGL(gram_partials_kernel, dim3(unsigned(maxc), unsigned(job.nfac)), dim3(256),
                     lds, s, job, r);
  return hipGetLastError();
}

hipError_t launch_hadamard(const HadamardJob& job, int r, float* G32, double* G64,
                           hipStream_t s) {
  const int blocks = int(ceil_div(int64_t(r) * r, 256));
  hipLaunchKernelGGL(hadamard_kernel, dim3(blocks), dim3(256), 0, s, job, r, G32, G64);
  return hipGetLastError();
}

}  // namespace ntf
