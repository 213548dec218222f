// Document build through the whitened moment tensor (Appendix D, the moment
// combination of Eq. (moment3) with the per-document terms of Eq. (td)).
//
// M3(W, W, W) is a sum of rank-1 terms of two shapes, x (x) x (x) x and
// x (x) x (x) y with their mode permutations, plus q (x) q (x) q.  With the
// index pairs i <= j as rows, every such sum over items t is one dense product
//   C[(i,j)][c] = sum_t x_t[i] x_t[j] B_t[c],
// whose columns c hold the item's weighted x (the x^(x)3 terms), its weighted
// y (the x x y terms) and its weight alone (the second-order sums that the
// q terms need).  For small K (the whitened dimension) this costs about
// D K^3 / 2 multiply-adds on the matrix cores in FP64, where the route of
// Section 3.2 takes three real transforms of b points per document and sketch
// on the vector units; the K^3 tensor is then assembled from C and sketched
// by Eq. (1) like any dense tensor.
#pragma once

#include "kernels.hpp"

namespace tsk {

struct MomentArgs {
  const void* X;     // R[nitem][K]
  const void* Y;     // R[nitem][K] (HAS_Y) or null
  const double* cA;  // [nitem] weight of x^(x)3, times sa
  const double* cB;  // [nitem] weight of the second-order column, times sb
  double sa, sb, gam;
  int K, nitem, per;  // items per chunk (blockIdx.y)
  int np;             // pairs K (K + 1) / 2
  int ncol;           // columns: K + 1, or 2 K + 1 with HAS_Y
  int rows, ld;       // rows and row stride of one chunk's block of part
  double* part;       // [nchunk][rows][ld]
};

constexpr int kMomRT = 2;    // row tiles of 16 pairs per wave
constexpr int kMomCT = 7;    // column tiles of 16 per work-group
constexpr int kMomTI = 32;   // items staged in LDS at a time
constexpr int kMomRows = 4 * kMomRT * 16;  // pair rows per work-group (four waves)
constexpr int kMomCols = kMomCT * 16;
constexpr int kMomNX = (kMomTI * 128 + 255) / 256;  // staged values per thread for K <= 128

inline size_t moment_lds_bytes(int K, bool has_y) {
  return sizeof(double) * ((size_t)kMomTI * K * (has_y ? 2 : 1) + 2 * kMomTI);
}

// Pairs a <= b in column-major order: p = b (b + 1) / 2 + a, so that a block
// of consecutive rows has nearly one b.
__host__ __device__ inline int moment_pidx(int i, int j) {
  const int lo = i < j ? i : j, hi = i < j ? j : i;
  return hi * (hi + 1) / 2 + lo;
}
__device__ inline int moment_pair_b(int p) {
  int b = (int)((sqrt(8.0 * p + 1.0) - 1.0) * 0.5);
  while (b * (b + 1) / 2 > p) --b;
  while ((b + 1) * (b + 2) / 2 <= p) ++b;
  return b;
}

// Partial products of one chunk of items for a block of 128 pair rows and
// 112 columns: work-group (row block, column group) x chunk, four waves of
// 2 x 7 tiles; one MFMA step takes four items.  A[r][k] = x_t[a] x_t[b] for
// pair row r = (a, b) and item t = step + k, B[k][c] = B_t[c].  The x^(x)3
// columns c < K are needed only for c >= b (the tensor is symmetric, the
// assembly reads them with sorted indices), so a wave leaves out the column
// tiles below the smallest b of its rows.  Rows past np compute on pair
// (0, 0) and are never read back; left-out tiles are written as zeros, so
// every partial the chunk sums read is defined.  The next
// stage's items are loaded while the current one runs, and B is formed from
// the staged x (and y) at each step.
template <typename R, bool HAS_Y>
__global__ __launch_bounds__(256) void k_moment3(MomentArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int K = a.K, TK = kMomTI * K;
  double* xs = reinterpret_cast<double*>(lds_raw);  // [TI][K], then y [TI][K] (HAS_Y)
  double* ys = xs + TK;
  double* cs = ys + (HAS_Y ? TK : 0);               // [2][TI]: sa cA, sb cB
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ncg = (a.ncol + kMomCols - 1) / kMomCols;
  const int rb = blockIdx.x / ncg, cg = blockIdx.x % ncg;
  const int ntc = (a.ncol + 15) >> 4;  // column tiles in use overall
  const int c0 = cg * kMomCols;
  int pa[kMomRT], pb[kMomRT];
#pragma unroll
  for (int rt = 0; rt < kMomRT; ++rt) {
    const int p = rb * kMomRows + (wave * kMomRT + rt) * 16 + r16;
    pa[rt] = pb[rt] = 0;
    if (p < a.np) {
      pb[rt] = moment_pair_b(p);
      pa[rt] = p - pb[rt] * (pb[rt] + 1) / 2;
    }
  }
  // column tiles this wave computes (wave-uniform)
  const int p0 = rb * kMomRows + wave * kMomRT * 16;
  unsigned act = 0;
  if (p0 < a.np) {
    const int bmin = moment_pair_b(p0);
#pragma unroll
    for (int ct = 0; ct < kMomCT; ++ct) {
      const int g = cg * kMomCT + ct, last = 16 * g + 15;
      if (g < ntc && (last >= bmin || last >= K)) act |= 1u << ct;
    }
  }
  // column c of lane r16 in tile ct: B_t[c] = w xs[t K + off] with w = sa cA_t
  // on x columns and gam on y columns; sb cB_t in the second-order column; 0
  // past it
  int off[kMomCT];
  unsigned colx = 0, coly = 0, cols2 = 0;
#pragma unroll
  for (int ct = 0; ct < kMomCT; ++ct) {
    const int c = c0 + ct * 16 + r16;
    off[ct] = 0;
    if (c < K) {
      off[ct] = c;
      colx |= 1u << ct;
    } else if (HAS_Y && c < 2 * K) {
      off[ct] = TK + (c - K);
      coly |= 1u << ct;
    } else if (c == a.ncol - 1) {
      cols2 |= 1u << ct;
    }
  }
  const R* X = reinterpret_cast<const R*>(a.X);
  const R* Y = reinterpret_cast<const R*>(a.Y);
  const int i0 = blockIdx.y * a.per, i1 = min(a.nitem, i0 + a.per);
  const size_t lim = (size_t)i1 * K;
  R xr[kMomNX], yr[kMomNX];
  unsigned vmask = 0;  // staged values inside the chunk
  double cr = 0.0;
  bool cvalid = false;
  // Every load is issued unconditionally from a clamped address and its value
  // is masked only when it is written to LDS, so the loads of a stage are all
  // in flight together and are waited for at the next stage.
  auto fetch = [&](int s) {
    const size_t base = (size_t)s * K;
    vmask = 0;
#pragma unroll
    for (int u = 0; u < kMomNX; ++u) {
      const size_t g = base + min(tid + 256 * u, TK - 1);
      const size_t gc = g < lim ? g : lim - 1;
      xr[u] = X[gc];
      if (HAS_Y) yr[u] = Y[gc];
      vmask |= (g < lim ? 1u : 0u) << u;
    }
    const int it = s + (tid & (kMomTI - 1));
    cvalid = tid < 2 * kMomTI && it < i1;
    cr = (tid < kMomTI ? a.cA : a.cB)[cvalid ? it : i0];
  };
  mfma_f64x4 acc[kMomRT][kMomCT];
#pragma unroll
  for (int rt = 0; rt < kMomRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < kMomCT; ++ct) acc[rt][ct] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
  if (i0 < i1) fetch(i0);
  for (int s0 = i0; s0 < i1; s0 += kMomTI) {
    __syncthreads();  // the previous stage's readers are done
#pragma unroll
    for (int u = 0; u < kMomNX; ++u) {
      const int e = tid + 256 * u;
      const bool ok = (vmask >> u) & 1u;
      if (e < TK) {
        xs[e] = ok ? (double)xr[u] : 0.0;
        if (HAS_Y) ys[e] = ok ? (double)yr[u] : 0.0;
      }
    }
    if (tid < 2 * kMomTI) cs[tid] = cvalid ? (tid < kMomTI ? a.sa : a.sb) * cr : 0.0;
    if (s0 + kMomTI < i1) fetch(s0 + kMomTI);  // in flight during the products below
    __syncthreads();
    if (act == 0) continue;
    const int steps = min(kMomTI, i1 - s0);
    for (int st = 0; st < steps; st += 4) {
      const int t = st + kq;
      const double ca = cs[t], cb = cs[kMomTI + t];
      double A[kMomRT], Bv[kMomCT];
#pragma unroll
      for (int rt = 0; rt < kMomRT; ++rt) A[rt] = xs[t * K + pa[rt]] * xs[t * K + pb[rt]];
#pragma unroll
      for (int ct = 0; ct < kMomCT; ++ct) {
        const double v = xs[t * K + off[ct]];
        const double w = (colx >> ct) & 1u ? ca : ((coly >> ct) & 1u ? a.gam : 0.0);
        Bv[ct] = (cols2 >> ct) & 1u ? cb : w * v;
      }
#pragma unroll
      for (int ct = 0; ct < kMomCT; ++ct) {
        if (act & (1u << ct)) {
#pragma unroll
          for (int rt = 0; rt < kMomRT; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[rt], Bv[ct], acc[rt][ct], 0, 0, 0);
        }
      }
    }
  }
  double* out = a.part + (size_t)blockIdx.y * a.rows * a.ld;
#pragma unroll
  for (int rt = 0; rt < kMomRT; ++rt) {
    const int rbase = rb * kMomRows + (wave * kMomRT + rt) * 16;
#pragma unroll
    for (int ct = 0; ct < kMomCT; ++ct) {  // left-out tiles hold their zeros
      const int c = c0 + ct * 16 + r16;
#pragma unroll
      for (int v = 0; v < 4; ++v) out[(size_t)(rbase + kq + 4 * v) * a.ld + c] = acc[rt][ct][v];
    }
  }
}

// C[r][c] = sum over the chunks, in chunk order, for r < np, c < ncol.
__global__ void k_moment_reduce(const double* part, int nchunk, int rows, int ld, int np, int ncol,
                                double* C) {
  const size_t total = (size_t)np * ncol;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / ncol), c = (int)(e % ncol);
    double s = 0.0;
    for (int h = 0; h < nchunk; ++h) s += part[((size_t)h * rows + r) * ld + c];
    C[(size_t)r * ncol + c] = s;
  }
}

// The K^3 tensor from the document products Cd [np][K+1] (x^(x)3 sums, then
// the second-order column) and the word products Cw [np][2K+1] (w^(x)3
// sums, the w w R sums, the second-order column), with (a, b, c) the sorted
// (i, j, k) and S2[p] = Cd[p][K] + Cw[p][2K]:
//   T[i][j][k] = (Cd[ab][c] + Cw[ab][c] + Cw[ij][K+k] + Cw[ik][K+j] + Cw[jk][K+i]
//                 + S2[ij] q[k] + S2[ik] q[j] + S2[jk] q[i]) / D + c q[i] q[j] q[k].
__global__ void k_moment_assemble(const double* Cd, const double* Cw, const double* q, const double* deff,
                                  double c3, int K, double* T) {
  const double D = deff[0];
  const double invD = D > 0.0 ? 1.0 / D : 0.0;
  const int ncd = K + 1, ncw = 2 * K + 1;
  const size_t total = (size_t)K * K * K;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(e % K), j = (int)((e / K) % K), i = (int)(e / ((size_t)K * K));
    const int lo = min(i, min(j, k)), hi = max(i, max(j, k)), mid = i + j + k - lo - hi;
    const int pab = moment_pidx(lo, mid);
    const int pij = moment_pidx(i, j), pik = moment_pidx(i, k), pjk = moment_pidx(j, k);
    const double s2ij = Cd[(size_t)pij * ncd + K] + Cw[(size_t)pij * ncw + 2 * K];
    const double s2ik = Cd[(size_t)pik * ncd + K] + Cw[(size_t)pik * ncw + 2 * K];
    const double s2jk = Cd[(size_t)pjk * ncd + K] + Cw[(size_t)pjk * ncw + 2 * K];
    const double r = Cd[(size_t)pab * ncd + hi] + Cw[(size_t)pab * ncw + hi] + Cw[(size_t)pij * ncw + K + k] +
                     Cw[(size_t)pik * ncw + K + j] + Cw[(size_t)pjk * ncw + K + i];
    const double qs = s2ij * q[k] + s2ik * q[j] + s2jk * q[i];
    T[e] = (r + qs) * invD + c3 * q[i] * q[j] * q[k];
  }
}

}  // namespace tsk
