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

// Y = M2 X (rows w, K <= 128 columns); grid over words, 128 threads.  Four
// documents per step, with four partial sums, keep four rows of P in flight.
__global__ __launch_bounds__(128) void k_lda_m2_apply(const int32_t* sdoc, const int32_t* scnt,
                                                      const int32_t* colptr, const double* P, const double* cpd,
                                                      const double* invm, const double* X, const double* q,
                                                      const double* deff, double alpha0, int V, int K, double* Y) {
  const double Dk = deff[0];
  const double inv = Dk > 0.0 ? 1.0 / Dk : 0.0;
  const double a = alpha0 / (alpha0 + 1.0);
  const int k = threadIdx.x;
  const int kc = k < K ? k : 0;  // lanes past K read column 0 and discard it
  for (int w = blockIdx.x; w < V; w += gridDim.x) {
    const int lo = colptr[w], hi = colptr[w + 1];
    const double xw = X[(size_t)w * K + kc];
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, m1 = 0.0;
    int e = lo;
    for (; e + 4 <= hi; e += 4) {
      int d[4];
      double n[4], p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        d[u] = sdoc[e + u];
        n[u] = (double)scnt[e + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = P[(size_t)d[u] * K + kc];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        m1 += invm[d[u]] * n[u];
        acc[u] += cpd[d[u]] * n[u] * (p[u] - xw);
      }
    }
    for (; e < hi; ++e) {
      const int d = sdoc[e];
      const double n = (double)scnt[e];
      m1 += invm[d] * n;
      acc[0] += cpd[d] * n * (P[(size_t)d * K + kc] - xw);
    }
    if (k < K) Y[(size_t)w * K + k] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) * inv - a * (m1 * inv) * q[k];
  }
}

// G[r][c] = sum_w X[w][r] Y[w][c] (X, Y: [V][K]); grid (K, K), 256 threads.
__global__ __launch_bounds__(256) void k_gram2(const double* X, const double* Y, double* G, int V, int K) {
  __shared__ double red[4];
  const int r = blockIdx.x, c = blockIdx.y;
  double s = 0.0;
  for (int w = threadIdx.x; w < V; w += 256) s += X[(size_t)w * K + r] * Y[(size_t)w * K + c];
  const double g = block_sum<256>(s, red);
  if (threadIdx.x == 0) G[(size_t)r * K + c] = g;
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

}  // namespace tsk
