// Row-chunk partial Grams shared by the standalone Gram kernel and the A-HALS epilogue.
// Both must produce bit-identical partials for the same rows (the solver's Gram cache is
// filled by either), so the chunking and the summation order live here only.
#pragma once

#include "ntf_internal.h"

namespace ntf {

// Row layout of the A-HALS kernel: kHalsRowWaves waves own rows (a fourth wave runs the
// stopping rule, on a SIMD of its own); a row group of 16 lanes (r <= 32) or of a whole
// wave (r <= 128) owns a row; NR rows per group are processed together, NR as small as
// keeps the grid within 256 workgroups. The rows of one workgroup are also one Gram chunk.
constexpr int kHalsRowWaves = 3;
__host__ __device__ inline int hals_rows_interleaved(int r, int64_t rows) {
  const int64_t per_nr = kHalsRowWaves * (r <= 32 ? 4 : 1);  // rows per workgroup, NR = 1
  for (int nr = 1; nr < 4; nr *= 2)
    if ((rows + per_nr * nr - 1) / (per_nr * nr) <= 256) return nr;
  return 4;
}
__host__ __device__ inline int gram_chunk_rows(int r, int64_t rows) {
  return kHalsRowWaves * (r <= 32 ? 4 : 1) * hals_rows_interleaved(r, rows);
}

// out[p * r + q] = sum_{i < nrows} rows[i * r + p] * rows[i * r + q] in float64, rows taken
// in order (products of float32 values are exact in float64, so neither the tiling nor the
// use of fused multiply-adds changes the bits). `rows` is in LDS; all threads of the block
// take part, each owning T x T tiles of entries (tile t = threadIdx.x + k * blockDim.x);
// `out` is global and may be NULL. Returns the thread's share of
// sum_{p,q} M[p, q] out[p, q] for the optional float64 r x r matrix M (global), else 0.
// With PRE, the M entries of the thread's first tile come from `mfirst` (loaded early by
// the caller with gram_tile_m).
template <int T>
__device__ inline void gram_tile_m(const double* M, int r, int tile, double (&m)[T][T]) {
  const int nt = (r + T - 1) / T;
  const int p0 = (tile / nt) * T;
  const int q0 = (tile - (tile / nt) * nt) * T;
  // loads at clamped indices, then a select (no branch per load)
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const double v = M ? M[min(p0 + a, r - 1) * r + min(q0 + b, r - 1)] : 0.0;
      m[a][b] = (tile < nt * nt && p0 + a < r && q0 + b < r) ? v : 0.0;
    }
}

// U > 1: the row loop runs in blocks of U rows whose LDS loads are all in flight at once
// (rows past nrows add exact zeros, so the sums are the same); U = 1: a plain loop.
template <int T, bool PRE, int U = 1>
__device__ inline double chunk_gram_tiles(const float* rows, int nrows, int r, double* out,
                                          const double* M, const double (&mfirst)[T][T]) {
  const int nt = (r + T - 1) / T;
  double dot = 0.0;
  for (int tile = threadIdx.x; tile < nt * nt; tile += blockDim.x) {
    const int p0 = (tile / nt) * T;
    const int q0 = (tile - (tile / nt) * nt) * T;
    double m[T][T];
    if (PRE && tile == int(threadIdx.x)) {
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) m[a][b] = mfirst[a][b];
    } else {
      gram_tile_m<T>(M, r, tile, m);
    }
    double acc[T][T];
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b) acc[a][b] = 0.0;
    for (int i0 = 0; i0 < nrows; i0 += U) {
      float vp[U][T], vq[U][T];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // loads at clamped indices, then a select: conditional loads would become branches
        // that wait for each load in turn
        const float* row = rows + min(i0 + u, nrows - 1) * r;
#pragma unroll
        for (int a = 0; a < T; ++a) {
          vp[u][a] = row[min(p0 + a, r - 1)];
          vq[u][a] = row[min(q0 + a, r - 1)];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = i0 + u < nrows;
        double xp[T], xq[T];
#pragma unroll
        for (int a = 0; a < T; ++a) {
          xp[a] = live && p0 + a < r ? double(vp[u][a]) : 0.0;
          xq[a] = live && q0 + a < r ? double(vq[u][a]) : 0.0;
        }
#pragma unroll
        for (int a = 0; a < T; ++a)
#pragma unroll
          for (int b = 0; b < T; ++b) acc[a][b] = fma(xp[a], xq[b], acc[a][b]);
      }
    }
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b)
        if (p0 + a < r && q0 + b < r) {
          if (out) out[(p0 + a) * r + q0 + b] = acc[a][b];
          dot = fma(m[a][b], acc[a][b], dot);
        }
  }
  return dot;
}

// G = Hadamard product over the job's factors of their Grams (each the sum of its chunk
// partials in chunk order), as float32 and/or float64, and the reset of `nslots` inner
// solver wait slots to the sentinel; this block is number blk of nblk doing the work.
__device__ inline void hadamard_work(const HadamardJob& job, int r, float* G32, double* G64,
                                     double* slots, int64_t nslots, int64_t blk, int64_t nblk) {
  const int64_t tid = blk * blockDim.x + threadIdx.x;
  const int rr = r * r;
  // four consecutive threads per entry: thread q sums chunks q, q + 4, ... in order (up to
  // sixteen loads in flight), then the four sums are combined as (s0 + s1) + (s2 + s3) by
  // two exchanges (a + b and b + a are the same bits, so all four get the same value)
  const int q = int(tid & 3);
  const int64_t nq = (nblk * blockDim.x) >> 2;
  const bool restart = job.st != nullptr && job.st->restart != 0;
  for (int64_t e64 = tid >> 2; e64 < rr; e64 += nq) {
    const int e = int(e64);
    double g = 1.0;
    for (int f = 0; f < job.nfac; ++f) {
      double s = 0.0;
      const double* part = (restart && job.part_new[f]) ? job.part_new[f] : job.part[f];
      const int64_t nc = job.nchunks[f];
      for (int64_t c0 = 0; c0 < nc; c0 += 64) {
        double v[16];
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          const int64_t c = c0 + q + 4 * t;
          v[t] = part[(c < nc ? c : 0) * rr + e];
        }
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (c0 + q + 4 * t < nc) s += v[t];
      }
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      g *= s;
    }
    if (q == 0) {
      if (G32) G32[e] = float(g);
      if (G64) G64[e] = g;
    }
  }
  for (int64_t e = tid; e < nslots; e += nblk * blockDim.x)
    slots[e] = __longlong_as_double(-1ll);
}

// Both chunk Grams of two row blocks of the same shape in one pass (the A-HALS epilogue:
// new and extrapolated rows): each entry is summed exactly as chunk_gram_tiles sums it, so
// the partials are bit-identical to two separate calls. Returns the share of
// sum M .* out_a (as chunk_gram_tiles does for rows_a).
template <int T, bool PRE, int U>
__device__ inline double chunk_gram2_tiles(const float* rows_a, const float* rows_b,
                                           int nrows, int r, double* out_a, double* out_b,
                                           const double* M, const double (&mfirst)[T][T]) {
  const int nt = (r + T - 1) / T;
  double dot = 0.0;
  for (int tile = threadIdx.x; tile < nt * nt; tile += blockDim.x) {
    const int p0 = (tile / nt) * T;
    const int q0 = (tile - (tile / nt) * nt) * T;
    double m[T][T];
    if (PRE && tile == int(threadIdx.x)) {
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) m[a][b] = mfirst[a][b];
    } else {
      gram_tile_m<T>(M, r, tile, m);
    }
    double acc[2][T][T];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b) acc[h][a][b] = 0.0;
    for (int i0 = 0; i0 < nrows; i0 += U) {
      float vp[2][U][T], vq[2][U][T];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // loads at clamped indices, then a select (no branch per load)
          const float* row = (h ? rows_b : rows_a) + min(i0 + u, nrows - 1) * r;
#pragma unroll
          for (int a = 0; a < T; ++a) {
            vp[h][u][a] = row[min(p0 + a, r - 1)];
            vq[h][u][a] = row[min(q0 + a, r - 1)];
          }
        }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = i0 + u < nrows;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double xp[T], xq[T];
#pragma unroll
          for (int a = 0; a < T; ++a) {
            xp[a] = live && p0 + a < r ? double(vp[h][u][a]) : 0.0;
            xq[a] = live && q0 + a < r ? double(vq[h][u][a]) : 0.0;
          }
#pragma unroll
          for (int a = 0; a < T; ++a)
#pragma unroll
            for (int b = 0; b < T; ++b) acc[h][a][b] = fma(xp[a], xq[b], acc[h][a][b]);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b)
        if (p0 + a < r && q0 + b < r) {
          const int e = (p0 + a) * r + q0 + b;
          if (out_a) out_a[e] = acc[0][a][b];
          if (out_b) out_b[e] = acc[1][a][b];
          dot = fma(m[a][b], acc[0][a][b], dot);
        }
  }
  return dot;
}

// tile edge used for rank r
__host__ __device__ constexpr int gram_tile_edge(int r) { return r <= 32 ? 2 : 4; }

__device__ inline double chunk_gram(const float* rows, int nrows, int r, double* out,
                                    const double* M = nullptr) {
  const double z2[2][2] = {};
  const double z4[4][4] = {};
  return r <= 32 ? chunk_gram_tiles<2, false>(rows, nrows, r, out, M, z2)
                 : chunk_gram_tiles<4, false>(rows, nrows, r, out, M, z4);
}

}  // namespace ntf
