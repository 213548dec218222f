// Fast spectral LDA (Appendix D, Algorithm 3): the whitening from the
// empirical second moment and the recovery of the model from the CP
// decomposition of the whitened third moment.
//
// M2 = E[x1 (x) x2] - alpha0/(alpha0+1) M1 (x) M1 (Eq. (moment2)) with the
// per-document estimates (n n^T - diag n)/(m (m-1)) averaged over the
// documents of at least three words.  M2 is never formed: M2 X for a V x K
// block X is, row w,
//   (1/D) sum_{d containing w} n_dw (p_d - X[w]) / (m_d (m_d - 1))
//   - alpha0/(alpha0+1) M1[w] (M1^T X),       p_d = X^T n_d,
// over the documents of word w in document order (a stable sort by word).
// The truncated SVD is a randomized subspace iteration on such products.
#pragma once

#include "kernels.hpp"

namespace tsk {

// wk[d] = (w0[d], w1[d]): two per-document weights in one 16-byte word, so
// that a document costs one load of them, not two (the weights (c'_d, 1/m_d)
// of M2 X here, (c_d, c'_d) of the document build's per-word sums).
__global__ void k_pack_doc_weights(const double* w0, const double* w1, int D, double2* wk) {
  for (int d = blockIdx.x * blockDim.x + threadIdx.x; d < D; d += gridDim.x * blockDim.x)
    wk[d] = make_double2(w0[d], w1[d]);
}

// Y = M2 X (rows w, K <= 128 columns); one wave per word, two columns per
// lane (k and k + 64).  Sixteen documents per step, with as many partial sums
// per column, keep 32 loads of P in flight per lane, and the next step's
// document indices are loaded with this step's rows.  wk: the packed
// per-document weights (c'_d, 1/m_d) of k_pack_doc_weights.
__global__ __launch_bounds__(64) void k_lda_m2_apply(const int32_t* sdoc, const int32_t* scnt,
                                                     const int32_t* colptr, const double* P, const double2* wk,
                                                     const double* X, const double* q, const double* deff,
                                                     double alpha0, int V, int K, double* Y) {
  constexpr int U = 16, CPT = 2;
  const double Dk = deff[0];
  const double inv = Dk > 0.0 ? 1.0 / Dk : 0.0;
  const double a = alpha0 / (alpha0 + 1.0);
  int kc[CPT];
  bool kv[CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int k = (int)threadIdx.x + j * 64;
    kv[j] = k < K;
    kc[j] = kv[j] ? k : 0;  // lanes past K read column 0 and discard it
  }
  for (int w = blockIdx.x; w < V; w += gridDim.x) {
    const int lo = colptr[w], hi = colptr[w + 1];
    double xw[CPT], acc[CPT][U], m1 = 0.0;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      xw[j] = X[(size_t)w * K + kc[j]];
#pragma unroll
      for (int u = 0; u < U; ++u) acc[j][u] = 0.0;
    }
    int dn[U], nn[U];
    auto load_idx = [&](int e0) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        dn[u] = sdoc[e0 + u];
        nn[u] = scnt[e0 + u];
      }
    };
    int e = lo;
    if (e + U <= hi) load_idx(e);
    for (; e + U <= hi; e += U) {
      int d[U];
      double n[U], p[CPT][U], c[U], im[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        d[u] = dn[u];
        n[u] = (double)nn[u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int j = 0; j < CPT; ++j) p[j][u] = P[(size_t)d[u] * K + kc[j]];
        const double2 wd = wk[d[u]];
        c[u] = wd.x;
        im[u] = wd.y;
      }
      if (e + 2 * U <= hi) load_idx(e + U);  // the next step's indices, with this step's rows
#pragma unroll
      for (int u = 0; u < U; ++u) {
        m1 += im[u] * n[u];
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[j][u] += c[u] * n[u] * (p[j][u] - xw[j]);
      }
    }
    for (; e < hi; ++e) {
      const int d = sdoc[e];
      const double n = (double)scnt[e];
      const double2 wd = wk[d];
      m1 += wd.y * n;
#pragma unroll
      for (int j = 0; j < CPT; ++j) acc[j][0] += wd.x * n * (P[(size_t)d * K + kc[j]] - xw[j]);
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      // the partial sums pairwise, in a fixed order
#pragma unroll
      for (int h = 1; h < U; h *= 2)
#pragma unroll
        for (int u = 0; u < U; u += 2 * h) acc[j][u] += acc[j][u + h];
      if (kv[j]) Y[(size_t)w * K + kc[j]] = acc[j][0] * inv - a * (m1 * inv) * q[kc[j]];
    }
  }
}

// Partial Gram products over word chunks: part[z][r][c] = sum over the words
// w of chunk z of X[w][r] Y[w][c] (X, Y: [V][K]); work-group (16 x 16 tile of
// G, chunk z), the chunk's rows staged 64 at a time in LDS from clamped
// addresses (all loads in flight together), each entry summed in word order.
__global__ __launch_bounds__(256) void k_gram2(const double* X, const double* Y, double* part, int V, int K,
                                               int Z) {
  constexpr int TW = 64;
  __shared__ double xs[TW][16], ys[TW][16];
  const int r0 = blockIdx.x * 16, c0 = blockIdx.y * 16, z = blockIdx.z;
  const int per = (V + Z - 1) / Z, w_lo = z * per, w_hi = min(V, w_lo + per);
  const int i = threadIdx.x & 15, j = threadIdx.x >> 4;
  double s = 0.0;
  for (int w0 = w_lo; w0 < w_hi; w0 += TW) {
    __syncthreads();  // the previous stage's readers are done
    double vx[TW * 16 / 256], vy[TW * 16 / 256];
#pragma unroll
    for (int u = 0; u < TW * 16 / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int w = min(w0 + (e >> 4), V - 1), q = e & 15;
      vx[u] = X[(size_t)w * K + min(r0 + q, K - 1)];
      vy[u] = Y[(size_t)w * K + min(c0 + q, K - 1)];
    }
#pragma unroll
    for (int u = 0; u < TW * 16 / 256; ++u) {
      const int e = threadIdx.x + 256 * u;
      const bool ok = w0 + (e >> 4) < w_hi;
      xs[e >> 4][e & 15] = ok ? vx[u] : 0.0;
      ys[e >> 4][e & 15] = ok ? vy[u] : 0.0;
    }
    __syncthreads();
    const int nw = min(TW, w_hi - w0);
    for (int t = 0; t < nw; ++t) s += xs[t][i] * ys[t][j];
  }
  const int r = r0 + i, c = c0 + j;
  if (r < K && c < K) part[((size_t)z * K + r) * K + c] = s;
}

// G = the sum of the chunk partials, in chunk order.
__global__ void k_gram2_sum(const double* part, int Z, int K, double* G) {
  const size_t kk = (size_t)K * K;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < kk; e += (size_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < Z; ++z) s += part[(size_t)z * kk + e];
    G[e] = s;
  }
}

// Eigenpairs of the symmetric part of the k x k matrix G (k <= 100), one
// work-group of 256 threads with the matrix and the eigenvectors in dynamic
// LDS (jacobi_sweeps).  E[r][j] is component r of eigenvector j, d[j] its
// eigenvalue.
__global__ __launch_bounds__(256) void k_jacobi_eig(const double* G, int k, double* E, double* d) {
  extern __shared__ __align__(16) unsigned char lds[];
  double* A = reinterpret_cast<double*>(lds);
  double* Ev = A + (size_t)k * k;
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (int e = tid; e < k * k; e += 256) {
    const int r = e / k, c = e % k;
    A[e] = 0.5 * (G[(size_t)r * k + c] + G[(size_t)c * k + r]);
    Ev[e] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_sweeps(A, Ev, k, red);
  for (int e = tid; e < k * k; e += 256) E[e] = Ev[e];
  for (int j = tid; j < k; j += 256) d[j] = A[j * k + j];
}

// Q = Y E diag(1/sqrt(d)) (columns with d <= 1e-12 max d set to zero): an
// orthonormal basis of range(Y) from the eigenpairs of Y^T Y.  grid over
// rows, 128 threads (column j per thread).
__global__ __launch_bounds__(128) void k_orth_apply(const double* Y, const double* E, const double* d, double* Q,
                                                    int V, int K) {
  __shared__ double row[128];
  double dmax = 0.0;
  for (int j = 0; j < K; ++j) dmax = fmax(dmax, d[j]);
  const int j = threadIdx.x;
  const double dj = j < K ? d[j] : 0.0;
  const double s = (j < K && dj > 1e-12 * dmax) ? 1.0 / sqrt(dj) : 0.0;
  for (int w = blockIdx.x; w < V; w += gridDim.x) {
    __syncthreads();
    if (j < K) row[j] = Y[(size_t)w * K + j];
    __syncthreads();
    if (j < K) {
      double acc = 0.0;
      for (int c = 0; c < K; ++c) acc += row[c] * E[(size_t)c * K + j];
      Q[(size_t)w * K + j] = acc * s;
    }
  }
}

// W[w][r] = sum_c Q[w][c] E[c][j] / sqrt|d_j| and sigma[r] = |d_j| with r the
// rank of eigenpair j by decreasing |d| (ties: lower j first).
__global__ __launch_bounds__(128) void k_whiten_out(const double* Q, const double* E, const double* d, double* W,
                                                    double* sigma, int V, int K) {
  __shared__ double row[128];
  __shared__ int rank[128];
  const int j = threadIdx.x;
  if (j < K) {
    const double aj = fabs(d[j]);
    int r = 0;
    for (int i = 0; i < K; ++i) {
      const double ai = fabs(d[i]);
      r += (ai > aj) || (ai == aj && i < j);
    }
    rank[j] = r;
    if (blockIdx.x == 0) sigma[r] = aj;
  }
  const double s = j < K ? 1.0 / sqrt(fabs(d[j])) : 0.0;
  for (int w = blockIdx.x; w < V; w += gridDim.x) {
    __syncthreads();
    if (j < K) row[j] = Q[(size_t)w * K + j];
    __syncthreads();
    if (j < K) {
      double acc = 0.0;
      for (int c = 0; c < K; ++c) acc += row[c] * E[(size_t)c * K + j];
      W[(size_t)w * K + rank[j]] = acc * s;
    }
  }
}

// t_i = G^+ u_i (G = W^T W through its eigenpairs E, d; eigenvalues below
// 1e-12 of the largest dropped); grid = k, 128 threads.
__global__ __launch_bounds__(128) void k_lda_tvec(const double* E, const double* d, const double* U, int K,
                                                  double* t) {
  __shared__ double y[128];
  const int i = blockIdx.x, j = threadIdx.x;
  double dmax = 0.0;
  for (int l = 0; l < K; ++l) dmax = fmax(dmax, fabs(d[l]));
  // y = diag(1/d) E^T u_i
  if (j < K) {
    double acc = 0.0;
    for (int c = 0; c < K; ++c) acc += E[(size_t)c * K + j] * U[(size_t)i * K + c];
    y[j] = fabs(d[j]) > 1e-12 * dmax ? acc / d[j] : 0.0;
  }
  __syncthreads();
  if (j < K) {
    double acc = 0.0;
    for (int l = 0; l < K; ++l) acc += E[(size_t)j * K + l] * y[l];
    t[(size_t)i * K + j] = acc;
  }
}

// mu[i][w] = (alpha0+2)/2 lam_i sum_j W[w][j] t_i[j] (= (W^+)^T v_i scaled),
// alpha[i] = 4 alpha0 (alpha0+1) / ((alpha0+2)^2 lam_i^2); grid (ceil(V/256), k).
__global__ __launch_bounds__(256) void k_lda_mu(const double* W, const double* t, const double* lam,
                                                double alpha0, int V, int K, double* mu, double* alpha) {
  const int i = blockIdx.y;
  const int w = blockIdx.x * 256 + threadIdx.x;
  const double l = lam[i];
  if (blockIdx.x == 0 && threadIdx.x == 0)
    alpha[i] = 4.0 * alpha0 * (alpha0 + 1.0) / ((alpha0 + 2.0) * (alpha0 + 2.0) * l * l);
  if (w >= V) return;
  double acc = 0.0;
  for (int j = 0; j < K; ++j) acc += W[(size_t)w * K + j] * t[(size_t)i * K + j];
  mu[(size_t)i * V + w] = 0.5 * (alpha0 + 2.0) * l * acc;
}

// ---------------------------------------------------------------------------
// Held-out likelihood of a topic model (Section 5.2)
// ---------------------------------------------------------------------------

// Fixed-order sums and an argmin over a 256-thread work-group (red: 8 doubles
// and 8 ints of LDS); every thread returns the result.  The leading barrier
// keeps a previous call's readers of red safe.
__device__ inline double hl_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}
__device__ inline void hl_argmin(double& v, int& k, double* red, int* redi) {
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int ok = __shfl_xor(k, o);
    if (ov < v || (ov == v && ok < k)) {
      v = ov;
      k = ok;
    }
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = v;
    redi[threadIdx.x >> 6] = k;
  }
  __syncthreads();
  v = red[0];
  k = redi[0];
  for (int w = 1; w < 4; ++w)
    if (red[w] < v || (red[w] == v && redi[w] < k)) {
      v = red[w];
      k = redi[w];
    }
}

// LDS words (doubles) of k_simplex_ls for K topics.
__host__ __device__ constexpr size_t simplex_ls_lds_words(int K) { return (size_t)K * K + 4 * (size_t)K + 8; }

// One work-group of 256 threads per document d: the mixing vector
//   pi = argmin { (1/2) pi^T G pi - c^T pi : pi >= 0, sum pi = 1 },
// G = Phi^T Phi, c = Phi^T n_d / m_d = P[d] / m_d, by the primal active-set
// method for convex quadratic programmes: on the free set F the KKT system of
// min (1/2) x^T G_FF x - c_F^T x, 1^T x = 1 is solved through the Cholesky
// factor of G_FF (x = y1 - nu y2 with G_FF y1 = c_F, G_FF y2 = 1,
// nu = (1^T y1 - 1) / 1^T y2); a non-negative x is taken, and the index held at
// zero with the most negative multiplier mu_k = (G pi - c)_k + nu (lowest index
// on ties) enters F unless every mu_k >= -1e-12 max diag G; otherwise the step
// towards x stops where the first weight reaches zero and that index leaves F.
// The start is the best vertex.  Then L_d = (1/m) sum_i n_i ln(Phi[w_i] . pi).
// A document with no words, or one not solved in max_iter steps, gets NaN.
__global__ __launch_bounds__(256) void k_simplex_ls(const double* G, const double* P, const int32_t* rowptr,
                                                    const int32_t* col, const int32_t* cnt, const double* Phi,
                                                    int D, int K, int max_iter, double* pi_out,
                                                    double* ll_out) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  double* Lf = reinterpret_cast<double*>(lds_raw);  // nf x nf Cholesky factor
  double* pi = Lf + (size_t)K * K;
  double* c = pi + K;
  double* x = c + K;
  int* fidx = reinterpret_cast<int*>(x + K);          // K ints
  __shared__ double red[8];
  __shared__ int redi[8];
  __shared__ double s_nu;
  __shared__ int s_nf;
  const int tid = threadIdx.x;
  // tolerance of the multipliers: relative to the largest diagonal entry of G
  double gd = 0.0;
  for (int k = tid; k < K; k += 256) gd = fmax(gd, G[(size_t)k * K + k]);
  for (int o = 32; o > 0; o >>= 1) gd = fmax(gd, __shfl_xor(gd, o));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = gd;
  __syncthreads();
  const double tol = 1e-12 * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  for (int d = blockIdx.x; d < D; d += gridDim.x) {
    const int lo = rowptr[d], hi = rowptr[d + 1];
    double mloc = 0.0;
    for (int e = lo + tid; e < hi; e += 256) mloc += (double)cnt[e];
    const double m = hl_sum(mloc, red);
    if (!(m > 0.0)) {
      for (int k = tid; k < K; k += 256) pi_out[(size_t)d * K + k] = 0.0;
      if (tid == 0) ll_out[d] = __builtin_nan("");
      continue;
    }
    for (int k = tid; k < K; k += 256) {
      c[k] = P[(size_t)d * K + k] / m;
      pi[k] = 0.0;
    }
    __syncthreads();
    // best vertex
    double bv = __builtin_inf();
    int bk = 0x7fffffff;
    for (int k = tid; k < K; k += 256) {
      const double v = 0.5 * G[(size_t)k * K + k] - c[k];
      if (v < bv) {
        bv = v;
        bk = k;
      }
    }
    hl_argmin(bv, bk, red, redi);
    if (tid == 0) {
      fidx[0] = bk;
      pi[bk] = 1.0;
      s_nf = 1;
    }
    __syncthreads();
    bool done = false;
    for (int it = 0; it < max_iter && !done; ++it) {
      const int nf = s_nf;
      // Cholesky factor of G_FF, right-looking, lower triangle
      for (int e = tid; e < nf * nf; e += 256) {
        const int r = e / nf, q = e - r * nf;
        Lf[e] = G[(size_t)fidx[r] * K + fidx[q]];
      }
      __syncthreads();
      for (int j = 0; j < nf; ++j) {
        if (tid == 0) Lf[j * nf + j] = sqrt(Lf[j * nf + j]);
        __syncthreads();
        for (int r = j + 1 + tid; r < nf; r += 256) Lf[r * nf + j] /= Lf[j * nf + j];
        __syncthreads();
        const int t = nf - j - 1;  // trailing block rows j+1 .. nf-1
        for (int e = tid; e < t * t; e += 256) {
          const int r = j + 1 + e / t, q = j + 1 + e % t;
          if (q <= r) Lf[r * nf + q] -= Lf[r * nf + j] * Lf[q * nf + j];
        }
        __syncthreads();
      }
      // G_FF y1 = c_F and G_FF y2 = 1 by substitution in wave 0: lane l keeps
      // y[l] and y[l + 64] in registers; each row's dot product is a butterfly
      // sum, so every lane has the new value and its owner keeps it.
      if (tid < 64) {
        double ya[2] = {0.0, 0.0}, yb[2] = {0.0, 0.0};
        for (int r = 0; r < nf; ++r) {   // L z = b
          double s1 = 0.0, s2 = 0.0;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = tid + 64 * h;
            if (j < r) {
              s1 += Lf[r * nf + j] * ya[h];
              s2 += Lf[r * nf + j] * yb[h];
            }
          }
          for (int o = 32; o > 0; o >>= 1) {
            s1 += __shfl_xor(s1, o);
            s2 += __shfl_xor(s2, o);
          }
          const double dr = Lf[r * nf + r];
          const double v1 = (c[fidx[r]] - s1) / dr, v2 = (1.0 - s2) / dr;
          if ((r & 63) == tid) {
            ya[r >> 6] = v1;
            yb[r >> 6] = v2;
          }
        }
        for (int r = nf - 1; r >= 0; --r) {   // L^T y = z
          double s1 = 0.0, s2 = 0.0;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int j = tid + 64 * h;
            if (j > r && j < nf) {
              s1 += Lf[j * nf + r] * ya[h];
              s2 += Lf[j * nf + r] * yb[h];
            }
          }
          for (int o = 32; o > 0; o >>= 1) {
            s1 += __shfl_xor(s1, o);
            s2 += __shfl_xor(s2, o);
          }
          const double dr = Lf[r * nf + r];
          const double z1 = __shfl(ya[r >> 6], r & 63), z2 = __shfl(yb[r >> 6], r & 63);
          const double v1 = (z1 - s1) / dr, v2 = (z2 - s2) / dr;
          if ((r & 63) == tid) {
            ya[r >> 6] = v1;
            yb[r >> 6] = v2;
          }
        }
        double a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (tid + 64 * h < nf) {
            a1 += ya[h];
            a2 += yb[h];
          }
        for (int o = 32; o > 0; o >>= 1) {
          a1 += __shfl_xor(a1, o);
          a2 += __shfl_xor(a2, o);
        }
        const double nu = (a1 - 1.0) / a2;
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (tid + 64 * h < nf) x[tid + 64 * h] = ya[h] - nu * yb[h];
        if (tid == 0) s_nu = nu;
      }
      __syncthreads();
      const double nu = s_nu;
      bool neg = false;
      for (int i = tid; i < nf; i += 256) neg |= x[i] < 0.0;
      const bool infeasible = hl_sum(neg ? 1.0 : 0.0, red) > 0.0;
      if (!infeasible) {
        for (int i = tid; i < nf; i += 256) pi[fidx[i]] = x[i];
        __syncthreads();
        // multipliers of the indices held at zero
        double mv = __builtin_inf();
        int mk = 0x7fffffff;
        for (int k = tid; k < K; k += 256) {
          if (pi[k] != 0.0) continue;
          bool in_f = false;
          for (int i = 0; i < nf; ++i) in_f |= fidx[i] == k;
          if (in_f) continue;
          double g = -c[k] + nu;
          for (int i = 0; i < nf; ++i) g += G[(size_t)k * K + fidx[i]] * pi[fidx[i]];
          if (g < mv) {
            mv = g;
            mk = k;
          }
        }
        hl_argmin(mv, mk, red, redi);
        if (!(mv < -tol)) {
          done = true;
        } else if (tid == 0) {
          fidx[nf] = mk;
          s_nf = nf + 1;
        }
      } else {
        // ratio test: the first free weight to reach zero on the way to x
        double rv = __builtin_inf();
        int ri = 0x7fffffff;
        for (int i = tid; i < nf; i += 256) {
          if (x[i] < 0.0) {
            const double cur = pi[fidx[i]];
            const double r = cur / (cur - x[i]);
            if (r < rv || (r == rv && fidx[i] < (ri < nf ? fidx[ri] : 0x7fffffff))) {
              rv = r;
              ri = i;
            }
          }
        }
        // ties broken by the lower topic index: compare (ratio, topic)
        int rk = ri < nf ? fidx[ri] : 0x7fffffff;
        hl_argmin(rv, rk, red, redi);
        for (int i = tid; i < nf; i += 256) {
          const int k = fidx[i];
          pi[k] = k == rk ? 0.0 : pi[k] + rv * (x[i] - pi[k]);
        }
        __syncthreads();
        if (tid == 0) {
          int pos = 0;
          while (fidx[pos] != rk) ++pos;
          fidx[pos] = fidx[nf - 1];
          s_nf = nf - 1;
        }
      }
      __syncthreads();
    }
    for (int k = tid; k < K; k += 256) pi_out[(size_t)d * K + k] = pi[k];
    double acc = 0.0;
    for (int e = lo + tid; e < hi; e += 256) {
      const double* row = Phi + (size_t)col[e] * K;
      double p = 0.0;
      for (int k = 0; k < K; ++k) p += row[k] * pi[k];
      acc += (double)cnt[e] * log(p);
    }
    const double ll = hl_sum(acc, red);
    if (tid == 0) ll_out[d] = done ? ll / m : __builtin_nan("");
    __syncthreads();
  }
}

}  // namespace tsk
