// Row-chunk partial Grams shared by the standalone Gram kernel and the A-HALS epilogue.
// Both must produce bit-identical partials for the same rows (the solver's Gram cache is
// filled by either), so the chunking and the summation order live here only.
#pragma once

#include "ntf_internal.h"

namespace ntf {

// Row layout of the A-HALS kernel: a row group of 16 lanes (r <= 32) or of a whole wave
// (r <= 128); NR rows per group are processed together, NR as small as keeps the grid
// within 256 workgroups of 4 waves. The rows of one workgroup are also one Gram chunk.
__host__ __device__ inline int hals_rows_interleaved(int r, int64_t rows) {
  const int64_t per_nr = 4 * (r <= 32 ? 4 : 1);  // rows per workgroup with NR = 1
  for (int nr = 1; nr < 4; nr *= 2)
    if ((rows + per_nr * nr - 1) / (per_nr * nr) <= 256) return nr;
  return 4;
}
__host__ __device__ inline int gram_chunk_rows(int r, int64_t rows) {
  return 4 * (r <= 32 ? 4 : 1) * hals_rows_interleaved(r, rows);
}

// out[p * r + q] = sum_{i < nrows} rows[i * r + p] * rows[i * r + q] in float64, rows taken
// in order (products of float32 values are exact in float64). `rows` is in LDS; all
// threads of the block take part; `out` is global.
__device__ inline void chunk_gram(const float* rows, int nrows, int r, double* out) {
  constexpr int kEPT = 8;
  const int rr = r * r;
  for (int base = 0; base < rr; base += blockDim.x * kEPT) {
    double acc[kEPT];
    int pp[kEPT], qq[kEPT];
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
      const int e = base + t * blockDim.x + threadIdx.x;
      acc[t] = 0.0;
      pp[t] = e < rr ? e / r : 0;
      qq[t] = e < rr ? e - (e / r) * r : 0;
    }
    for (int i = 0; i < nrows; ++i) {
      const float* row = rows + i * r;
#pragma unroll
      for (int t = 0; t < kEPT; ++t) acc[t] += double(row[pp[t]]) * double(row[qq[t]]);
    }
#pragma unroll
    for (int t = 0; t < kEPT; ++t) {
      const int e = base + t * blockDim.x + threadIdx.x;
      if (e < rr) out[e] = acc[t];
    }
  }
}

}  // namespace ntf
