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
constexpr int kMomCT = 8;    // column tiles of 16 per work-group
constexpr int kMomTI = 32;   // items staged in LDS at a time
constexpr int kMomRows = 4 * kMomRT * 16;  // pair rows per work-group (four waves)
constexpr int kMomCols = kMomCT * 16;

__host__ __device__ constexpr int moment_kpad(int K) { return K | 1; }  // odd stride: rows on other banks
inline size_t moment_lds_bytes(int K) {
  return sizeof(double) * (size_t)kMomTI * (size_t)(moment_kpad(K) + kMomCols);
}

// Pair p < np of the row-major enumeration of i <= j < K.
__device__ inline void moment_pair(int p, int K, int& i, int& j) {
  int r = p, ii = 0;
  while (r >= K - ii) {
    r -= K - ii;
    ++ii;
  }
  i = ii;
  j = ii + r;
}

// Partial products of one chunk of items for a block of 128 pair rows and
// 128 columns: work-group (row block, column group) x chunk, four waves of
// 2 x 8 tiles; one MFMA step takes four items.  A[r][k] = x_t[i] x_t[j] for
// pair row r and item t = step + k, B[k][c] = B_t[c].  Rows past np compute
// on pair (0, 0) and are never read back.
template <typename R, bool HAS_Y>
__global__ __launch_bounds__(256) void k_moment3(MomentArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int K = a.K, KP = moment_kpad(K);
  double* xs = reinterpret_cast<double*>(lds_raw);  // [TI][KP]
  double* bs = xs + kMomTI * KP;                    // [TI][128]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int ncg = (a.ncol + kMomCols - 1) / kMomCols;
  const int rb = blockIdx.x / ncg, cg = blockIdx.x % ncg;
  const int ntc = (a.ncol + 15) >> 4;  // column tiles in use overall
  const int c0 = cg * kMomCols;
  int pi[kMomRT], pj[kMomRT];
#pragma unroll
  for (int rt = 0; rt < kMomRT; ++rt) {
    const int p = rb * kMomRows + (wave * kMomRT + rt) * 16 + r16;
    pi[rt] = pj[rt] = 0;
    if (p < a.np) moment_pair(p, K, pi[rt], pj[rt]);
  }
  const R* X = reinterpret_cast<const R*>(a.X);
  const R* Y = reinterpret_cast<const R*>(a.Y);
  const int i0 = blockIdx.y * a.per, i1 = min(a.nitem, i0 + a.per);
  mfma_f64x4 acc[kMomRT][kMomCT];
#pragma unroll
  for (int rt = 0; rt < kMomRT; ++rt)
#pragma unroll
    for (int ct = 0; ct < kMomCT; ++ct) acc[rt][ct] = mfma_f64x4{0.0, 0.0, 0.0, 0.0};
  for (int s0 = i0; s0 < i1; s0 += kMomTI) {
    __syncthreads();  // the previous stage's readers are done
    for (int e = threadIdx.x; e < kMomTI * K; e += blockDim.x) {
      const int t = e / K, k = e - t * K, it = s0 + t;
      xs[t * KP + k] = it < i1 ? (double)X[(size_t)it * K + k] : 0.0;
    }
    for (int e = threadIdx.x; e < kMomTI * kMomCols; e += blockDim.x) {
      const int t = e / kMomCols, c = c0 + (e - t * kMomCols), it = s0 + t;
      double v = 0.0;
      if (it < i1) {
        if (c < K) v = a.sa * a.cA[it] * (double)X[(size_t)it * K + c];
        else if (HAS_Y && c < 2 * K) v = a.gam * (double)Y[(size_t)it * K + (c - K)];
        else if (c == a.ncol - 1) v = a.sb * a.cB[it];
      }
      bs[e] = v;
    }
    __syncthreads();
    const int steps = min(kMomTI, i1 - s0);
    for (int st = 0; st < steps; st += 4) {
      const int t = st + kq;
      double A[kMomRT];
#pragma unroll
      for (int rt = 0; rt < kMomRT; ++rt) A[rt] = xs[t * KP + pi[rt]] * xs[t * KP + pj[rt]];
#pragma unroll
      for (int ct = 0; ct < kMomCT; ++ct) {
        if (cg * kMomCT + ct < ntc) {
          const double Bv = bs[t * kMomCols + ct * 16 + r16];
#pragma unroll
          for (int rt = 0; rt < kMomRT; ++rt)
            acc[rt][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[rt], Bv, acc[rt][ct], 0, 0, 0);
        }
      }
    }
  }
  double* out = a.part + (size_t)blockIdx.y * a.rows * a.ld;
#pragma unroll
  for (int rt = 0; rt < kMomRT; ++rt) {
    const int rbase = rb * kMomRows + (wave * kMomRT + rt) * 16;
#pragma unroll
    for (int ct = 0; ct < kMomCT; ++ct) {
      if (cg * kMomCT + ct < ntc) {
        const int c = c0 + ct * 16 + r16;
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(size_t)(rbase + kq + 4 * v) * a.ld + c] = acc[rt][ct][v];
      }
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
// sums, the w w R sums, the second-order column):
//   T[i][j][k] = (Cd[ij][k] + Cw[ij][k] + Cw[ij][K+k] + Cw[ik][K+j] + Cw[jk][K+i]
//                 + S2[ij] q[k] + S2[ik] q[j] + S2[jk] q[i]) / D + c q[i] q[j] q[k],
// S2[p] = Cd[p][K] + Cw[p][2K], ij the pair index of (min, max).
__device__ __forceinline__ int moment_pidx(int i, int j, int K) {
  const int lo = min(i, j), hi = max(i, j);
  return lo * K - (lo * (lo - 1)) / 2 + (hi - lo);
}

__global__ void k_moment_assemble(const double* Cd, const double* Cw, const double* q, const double* deff,
                                  double c3, int K, double* T) {
  const double D = deff[0];
  const double invD = D > 0.0 ? 1.0 / D : 0.0;
  const int ncd = K + 1, ncw = 2 * K + 1;
  const size_t total = (size_t)K * K * K;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int k = (int)(e % K), j = (int)((e / K) % K), i = (int)(e / ((size_t)K * K));
    const int pij = moment_pidx(i, j, K), pik = moment_pidx(i, k, K), pjk = moment_pidx(j, k, K);
    const double* dij = Cd + (size_t)pij * ncd;
    const double* wij = Cw + (size_t)pij * ncw;
    const double s2ij = dij[K] + wij[2 * K];
    const double s2ik = Cd[(size_t)pik * ncd + K] + Cw[(size_t)pik * ncw + 2 * K];
    const double s2jk = Cd[(size_t)pjk * ncd + K] + Cw[(size_t)pjk * ncw + 2 * K];
    const double r = dij[k] + wij[k] + wij[K + k] + Cw[(size_t)pik * ncw + K + j] +
                     Cw[(size_t)pjk * ncw + K + i];
    const double qs = s2ij * q[k] + s2ik * q[j] + s2jk * q[i];
    T[e] = (r + qs) * invD + c3 * q[i] * q[j] * q[k];
  }
}

}  // namespace tsk
