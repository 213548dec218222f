// Device kernels of the sketched robust tensor power method (gfx950, wave64).
//
// Layouts (device):
//   hx  [B][3][n]  uint32  (h << 1) | (xi < 0): packed bucket and sign
//   hxs [B][3][n]  uint32  the same entries sorted by bucket (stable in i)
//   ord [B][3][n]  uint32  the index i of each sorted entry
//   spectra        cx<R>[B][b/2+1]  half spectrum of each of the B sketches
//   vectors        R[L][n]
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft.hpp"

namespace tsk {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// Sum over the work-group, returned to every thread.  `red` holds NT/64 doubles.
template <int NT>
__device__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = (threadIdx.x < NT / 64) ? red[threadIdx.x] : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if (threadIdx.x == 0) red[0] = s;
  }
  __syncthreads();
  double s = red[0];
  __syncthreads();
  return s;
}

// Median of the values held by lanes 0..B-1 of a wave (B <= 64), returned to
// every lane; must be called by all 64 lanes.  Ranks break ties by lane, so
// ranks are a permutation; for even B the two middle values are averaged.
template <typename T>
__device__ T wave_median(T val, int B) {
  const int lane = wave_lane();
  int rank = 0;
  for (int mm = 0; mm < B; ++mm) {
    T o = __shfl(val, mm);
    rank += (o < val) || (o == val && mm < lane);
  }
  const bool valid = lane < B;
  auto pick = [&](int r) -> T {
    unsigned long long mask = __ballot(valid && rank == r);
    int src = mask ? (__ffsll((unsigned long long)mask) - 1) : 0;
    T x = __shfl(val, src);
    return mask ? x : T(__builtin_nan(""));
  };
  if (B & 1) return pick((B - 1) / 2);
  T lo = pick(B / 2 - 1);
  T hi = pick(B / 2);
  return (lo + hi) * T(0.5);
}

// Deterministic count sketch of u into dst[bucket * stride + off]: the entries
// sharing a bucket are summed by one thread in increasing index order.
template <typename R, typename U>
__device__ void count_sketch_lds(R* dst, int stride, int off, const uint32_t* __restrict__ hxs,
                                 const uint32_t* __restrict__ ord, const U* __restrict__ u, int n,
                                 int nt) {
  for (int p = threadIdx.x; p < n; p += nt) {
    uint32_t e = hxs[p];
    const uint32_t bk = e >> 1;
    if (p > 0 && (hxs[p - 1] >> 1) == bk) continue;
    R acc = R(0);
    int q = p;
    while (true) {
      const R val = (R)u[ord[q]];
      acc += (e & 1u) ? -val : val;
      if (++q >= n) break;
      e = hxs[q];
      if ((e >> 1) != bk) break;
    }
    dst[(size_t)bk * stride + off] = acc;
  }
}

// Threads per work-group for a transform of length 2^logb.
constexpr int threads_for(int logb) { return logb >= 14 ? 1024 : (logb >= 13 ? 512 : 256); }

// ---------------------------------------------------------------------------
// Power step / evaluation, one work-group per (sketch m, restart tau).
// ---------------------------------------------------------------------------
template <typename R>
struct PowerArgs {
  const uint32_t* hx;
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B;
  const cx<R>* S;       // [B][b/2+1]
  const cx<R>* tw;      // [b]
  const R* Uin;         // [L][n]
  R* Uout;              // [L][n]
  R* V;                 // [L][B][n]
  double* lam_per;      // [L][B]  (evaluate)
  double* lam_med;      // [L]     (evaluate)
  int32_t* flags;       // [L]     (power step; nullable)
  unsigned* counter;    // [L], zero between launches
  int tau0;             // first restart of this launch
  int mode;             // 0 = power step, 1 = evaluate T(u,u,u)
};

// P_k = S_k conj(F(s2)_k) conj(F(s3)_k) from the packed spectrum Z of s2 + i s3.
template <typename R>
__device__ __forceinline__ cx<R> spectrum_product(cx<R> Zk, cx<R> Zmk, cx<R> Sk) {
  const cx<R> zc = cconj(Zmk);
  const cx<R> s2 = cscale(cadd(Zk, zc), R(0.5));
  const cx<R> d = csub(Zk, zc);
  const cx<R> s3 = {R(0.5) * d.y, R(-0.5) * d.x};  // (Zk - conj Z_{b-k}) / (2i)
  return cmulc(Sk, cmul(s2, s3));
}

// Half-length packing for a real inverse transform: Y_k = E_k + i O_k with
// E_k = (X_k + conj X_{H-k})/2, O_k = (X_k - conj X_{H-k})/2 * conj(W^k).
template <typename R>
__device__ __forceinline__ cx<R> c2r_pack(cx<R> Xk, cx<R> XHk, cx<R> Wk) {
  const cx<R> c = cconj(XHk);
  const cx<R> E = cscale(cadd(Xk, c), R(0.5));
  const cx<R> O = cmulc(cscale(csub(Xk, c), R(0.5)), Wk);
  return {E.x - O.y, E.y + O.x};
}

template <typename R, int LOGB>
__global__ __launch_bounds__(threads_for(LOGB)) void k_power(PowerArgs<R> a) {
  constexpr int NT = threads_for(LOGB);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  __shared__ cx<R> buf[b];
  __shared__ double red[NT / 64];
  __shared__ int s_last;

  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const int tau = a.tau0 + blockIdx.y;
  const int n = a.n;
  const int B = a.B;
  const R* u = a.Uin + (size_t)tau * n;
  const size_t tb = (size_t)m * 3 * n;

  for (int t = tid; t < b; t += NT) buf[t] = cx<R>{R(0), R(0)};
  __syncthreads();
  // s2 into the real parts, s3 into the imaginary parts.
  count_sketch_lds<R, R>(reinterpret_cast<R*>(buf), 2, 0, a.hxs + tb + n, a.ord + tb + n, u, n, NT);
  count_sketch_lds<R, R>(reinterpret_cast<R*>(buf), 2, 1, a.hxs + tb + 2 * n, a.ord + tb + 2 * n, u,
                         n, NT);
  __syncthreads();
  fft_lds<R, LOGB, NT, false>(buf, a.tw, LOGB);

  // Product with the tensor's spectrum and packing for the half-length inverse.
  constexpr int NK = b / 4 + 1;
  constexpr int PK = (NK + NT - 1) / NT;
  const cx<R>* Sm = a.S + (size_t)m * (H + 1);
  cx<R> y0[PK], y1[PK];
#pragma unroll
  for (int q = 0; q < PK; ++q) {
    const int k = tid + q * NT;
    if (k < NK) {
      const int kk = H - k;
      const cx<R> Pk = spectrum_product(buf[k], buf[(b - k) & (b - 1)], Sm[k]);
      const cx<R> Pkk = spectrum_product(buf[kk], buf[H + k], Sm[kk]);
      y0[q] = c2r_pack(Pk, Pkk, a.tw[k]);
      y1[q] = c2r_pack(Pkk, Pk, a.tw[kk]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PK; ++q) {
    const int k = tid + q * NT;
    if (k < NK) {
      buf[k & (H - 1)] = y0[q];  // k = H/2 .. only k < H/2+1 <= H here
      if (k > 0 && k < b / 4) buf[H - k] = y1[q];
    }
  }
  __syncthreads();
  fft_lds<R, LOGB - 1, NT, true>(buf, a.tw, LOGB);

  // Read-off v_i = xi1(i) sbar[h1(i)], sbar = 2/b * (Re y, Im y) interleaved.
  const R scale = R(2) / R(b);
  const R* sbar = reinterpret_cast<const R*>(buf);
  const uint32_t* hx1 = a.hx + tb;
  R* Vrow = a.V + ((size_t)tau * B + m) * n;
  double acc = 0.0;
  for (int i = tid; i < n; i += NT) {
    const uint32_t e = hx1[i];
    const R val = sbar[e >> 1] * scale;
    const R v = (e & 1u) ? -val : val;
    Vrow[i] = v;
    acc += (double)u[i] * (double)v;
  }
  if (a.mode == 1) {
    const double lam = block_sum<NT>(acc, red);
    if (tid == 0) a.lam_per[(size_t)tau * B + m] = lam;
  }

  // The last of the B work-groups of this restart takes the median.
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (atomicAdd(&a.counter[tau], 1u) == (unsigned)(B - 1));
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  const int lane = wave_lane();
  const int wave = tid >> 6;
  constexpr int NW = NT / 64;
  if (a.mode == 1) {
    if (wave == 0) {
      const double x = lane < B ? __builtin_nontemporal_load(&a.lam_per[(size_t)tau * B + lane]) : 0.0;
      const double med = wave_median<double>(x, B);
      if (lane == 0) a.lam_med[tau] = med;
    }
  } else {
    R* uo = a.Uout + (size_t)tau * n;
    const R* vbase = a.V + (size_t)tau * B * n;
    double ss = 0.0;
    for (int i = wave; i < n; i += NW) {
      const R x = lane < B ? __builtin_nontemporal_load(&vbase[(size_t)lane * n + i]) : R(0);
      const R med = wave_median<R>(x, B);
      if (lane == 0) {
        uo[i] = med;
        ss += (double)med * (double)med;
      }
    }
    const double nrm = sqrt(block_sum<NT>(ss, red));
    const bool ok = nrm > 0.0 && nrm < __builtin_inf();
    if (lane == 0) {
      const R inv = ok ? R(1.0 / nrm) : R(0);
      for (int i = wave; i < n; i += NW) uo[i] = ok ? uo[i] * inv : u[i];
    }
    if (!ok && tid == 0 && a.flags) a.flags[tau] |= 1;
  }
  if (tid == 0) a.counter[tau] = 0u;
}

// ---------------------------------------------------------------------------
// FP64 rank-1 spectra: prod[r][m] = F(s1 u_r) o F(s2 u_r) o F(s3 u_r), optional
// lam_per[r][m] = <s^(m), s^(m)(u_r^(x)3)> by Parseval on the half spectrum.
// One work-group per (m, r); real transforms through half-length complex FFTs.
// ---------------------------------------------------------------------------
struct Rank1Args {
  const uint32_t* hx;
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B;
  const double* U;          // [c][n]
  const cx<double>* tw;     // [b]
  cx<double>* prod;         // [c][B][b/2+1]
  const cx<double>* S64;    // nullable: [B][b/2+1]
  double* lam_per;          // [c][B] when S64 != null
};

template <int LOGB>
__global__ __launch_bounds__(threads_for(LOGB - 1)) void k_rank1(Rank1Args a) {
  constexpr int NT = threads_for(LOGB - 1);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  __shared__ cx<double> buf[H];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const int r = blockIdx.y;
  const int n = a.n;
  const double* u = a.U + (size_t)r * n;
  cx<double>* P = a.prod + ((size_t)r * a.B + m) * (H + 1);
  for (int j = 0; j < 3; ++j) {
    const size_t tb = ((size_t)m * 3 + j) * n;
    for (int t = tid; t < H; t += NT) buf[t] = cx<double>{0.0, 0.0};
    __syncthreads();
    count_sketch_lds<double, double>(reinterpret_cast<double*>(buf), 1, 0, a.hxs + tb, a.ord + tb, u,
                                     n, NT);
    __syncthreads();
    fft_lds<double, LOGB - 1, NT, false>(buf, a.tw, LOGB);
    for (int k = tid; k <= H; k += NT) {
      const cx<double> Zk = buf[k & (H - 1)];
      const cx<double> Zc = cconj(buf[(H - k) & (H - 1)]);
      const cx<double> Xe = cscale(cadd(Zk, Zc), 0.5);
      const cx<double> d = csub(Zk, Zc);
      const cx<double> Xo = {0.5 * d.y, -0.5 * d.x};
      const cx<double> X = cadd(Xe, cmul(a.tw[k], Xo));
      P[k] = (j == 0) ? X : cmul(P[k], X);
    }
    __syncthreads();
  }
  if (a.S64) {
    const cx<double>* S = a.S64 + (size_t)m * (H + 1);
    double acc = 0.0;
    for (int k = tid; k <= H; k += NT) {
      const cx<double> s = S[k], p = P[k];
      const double w = (k == 0 || k == H) ? 1.0 : 2.0;
      acc += w * (s.x * p.x + s.y * p.y);
    }
    const double lam = block_sum<NT>(acc, red) / (double)b;
    if (tid == 0) a.lam_per[(size_t)r * a.B + m] = lam;
  }
}

// S64[m][k] += sum_r coef_r prod[r][m][k]; S32 = (float)S64.
// coef_r = sign * lam[r]; lam is a device array (e.g. lam_hat just computed).
__global__ void k_spec_update(cx<double>* S64, cx<float>* S32, const cx<double>* prod,
                              const double* lam, double sign, int c, int B, int H1) {
  const size_t total = (size_t)B * H1;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    cx<double> s = S64[e];
    for (int r = 0; r < c; ++r) {
      const double cf = sign * lam[r];
      const cx<double> p = prod[(size_t)r * total + e];
      s.x += cf * p.x;
      s.y += cf * p.y;
    }
    S64[e] = s;
    if (S32) S32[e] = cx<float>{(float)s.x, (float)s.y};
  }
}

// ---------------------------------------------------------------------------
// Time domain <-> half spectrum, FP64, one work-group per sketch.
// ---------------------------------------------------------------------------
template <int LOGB>
__global__ __launch_bounds__(threads_for(LOGB - 1)) void k_r2c64(const double* s_time,
                                                                   cx<double>* S64, cx<float>* S32,
                                                                   const cx<double>* tw, int accumulate) {
  constexpr int NT = threads_for(LOGB - 1);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  __shared__ cx<double> buf[H];
  const int m = blockIdx.x;
  const cx<double>* src = reinterpret_cast<const cx<double>*>(s_time + (size_t)m * b);
  for (int t = threadIdx.x; t < H; t += NT) buf[t] = src[t];
  __syncthreads();
  fft_lds<double, LOGB - 1, NT, false>(buf, tw, LOGB);
  cx<double>* S = S64 + (size_t)m * (H + 1);
  for (int k = threadIdx.x; k <= H; k += NT) {
    const cx<double> Zk = buf[k & (H - 1)];
    const cx<double> Zc = cconj(buf[(H - k) & (H - 1)]);
    const cx<double> Xe = cscale(cadd(Zk, Zc), 0.5);
    const cx<double> d = csub(Zk, Zc);
    const cx<double> Xo = {0.5 * d.y, -0.5 * d.x};
    cx<double> X = cadd(Xe, cmul(tw[k], Xo));
    if (accumulate) X = cadd(X, S[k]);
    S[k] = X;
    if (S32) S32[(size_t)m * (H + 1) + k] = cx<float>{(float)X.x, (float)X.y};
  }
}

template <int LOGB>
__global__ __launch_bounds__(threads_for(LOGB - 1)) void k_c2r64(const cx<double>* S64, double* s_time,
                                                                   const cx<double>* tw) {
  constexpr int NT = threads_for(LOGB - 1);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  __shared__ cx<double> buf[H];
  const int m = blockIdx.x;
  const cx<double>* S = S64 + (size_t)m * (H + 1);
  for (int k = threadIdx.x; k < H; k += NT) buf[k] = c2r_pack(S[k], S[H - k], tw[k]);
  __syncthreads();
  fft_lds<double, LOGB - 1, NT, true>(buf, tw, LOGB);
  double* dst = s_time + (size_t)m * b;
  const double scale = 2.0 / (double)b;
  for (int t = threadIdx.x; t < H; t += NT) {
    dst[2 * t] = buf[t].x * scale;
    dst[2 * t + 1] = buf[t].y * scale;
  }
}

// ---------------------------------------------------------------------------
// Dense build, Eq. (1).  Work-group (slab, group): the G sketches of `group`
// accumulate a contiguous slab of (i, j) fibres of T in LDS bins, then write
// the bins as one partial sum.  Each wave takes whole fibres T[i][j][:] with
// its lanes along k, so reads of T are coalesced.
// ---------------------------------------------------------------------------
template <typename TIn, typename TAcc>
struct BuildArgs {
  const TIn* T;
  int n, b, B, G;
  const uint32_t* hx;         // [B][3][n]
  long long pairs_per_slab;
  int nslab;
  TAcc* partial;              // [ngroups][nslab][G][b]
};

template <typename TIn, typename TAcc>
__global__ __launch_bounds__(256) void k_build_dense(BuildArgs<TIn, TAcc> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, b = a.b, G = a.G;
  const int g0 = blockIdx.y * G;
  const int Gc = min(G, a.B - g0);
  TAcc* bins = reinterpret_cast<TAcc*>(smem);
  uint32_t* tab = reinterpret_cast<uint32_t*>(bins + (size_t)G * b);  // [G][3][n]
  const int tid = threadIdx.x;
  for (int t = tid; t < G * b; t += blockDim.x) bins[t] = TAcc(0);
  for (int t = tid; t < Gc * 3 * n; t += blockDim.x) tab[t] = a.hx[(size_t)g0 * 3 * n + t];
  __syncthreads();

  const long long npairs = (long long)n * n;
  const long long p0 = (long long)blockIdx.x * a.pairs_per_slab;
  const long long p1 = min(npairs, p0 + a.pairs_per_slab);
  const int lane = tid & 63;
  const int nw = blockDim.x >> 6;
  const unsigned bmask = (unsigned)b - 1u;
  for (long long q = p0 + (tid >> 6); q < p1; q += nw) {
    const int i = (int)(q / n);
    const int j = (int)(q - (long long)i * n);
    const TIn* fib = a.T + q * n;
    for (int k = lane; k < n; k += 64) {
      const TAcc val = (TAcc)fib[k];
      for (int g = 0; g < Gc; ++g) {
        const uint32_t* tg = tab + (size_t)g * 3 * n;
        const uint32_t e1 = tg[i], e2 = tg[n + j], e3 = tg[2 * n + k];
        const unsigned t = ((e1 >> 1) + (e2 >> 1) + (e3 >> 1)) & bmask;
        atomicAdd(&bins[(size_t)g * b + t], ((e1 ^ e2 ^ e3) & 1u) ? -val : val);
      }
    }
  }
  __syncthreads();
  TAcc* out = a.partial + ((size_t)blockIdx.y * a.nslab + blockIdx.x) * (size_t)G * b;
  for (int t = tid; t < Gc * b; t += blockDim.x) out[t] = bins[t];
}

// s_time[m][t] = sum over slabs of the partial bins (FP64).
template <typename TAcc>
__global__ void k_build_reduce(const TAcc* partial, double* s_time, int b, int B, int G, int nslab) {
  const size_t total = (size_t)B * b;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / b);
    const int t = (int)(e - (size_t)m * b);
    const int grp = m / G, g = m - grp * G;
    const TAcc* p = partial + ((size_t)grp * nslab * G + g) * b + t;
    double s = 0.0;
    for (int sl = 0; sl < nslab; ++sl) s += (double)p[(size_t)sl * G * b];
    s_time[e] = s;
  }
}

// ---------------------------------------------------------------------------
// Selection and bookkeeping kernels (one work-group).
// ---------------------------------------------------------------------------
// tau* = argmax lam_med (lowest index on ties, non-finite never wins);
// u_hat = Ucand[tau*] / ||Ucand[tau*]|| in FP64.
template <typename R>
__global__ __launch_bounds__(256) void k_select(const double* lam_med, int L, const R* Ucand, int n,
                                                double* u_hat, double* U_out_row, int32_t* tau_out) {
  __shared__ double red[4];
  __shared__ int s_tau;
  if (threadIdx.x == 0) {
    int best = 0;
    double bv = -__builtin_inf();
    bool found = false;
    for (int t = 0; t < L; ++t) {
      const double x = lam_med[t];
      if (x == x && x > -__builtin_inf() && x < __builtin_inf() && (!found || x > bv)) {
        bv = x;
        best = t;
        found = true;
      }
    }
    s_tau = best;
    if (tau_out) *tau_out = best;
  }
  __syncthreads();
  const R* u = Ucand + (size_t)s_tau * n;
  double ss = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) ss += (double)u[i] * (double)u[i];
  const double nrm = sqrt(block_sum<256>(ss, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double x = (double)u[i] * inv;
    u_hat[i] = x;
    U_out_row[i] = x;
  }
}

// lam_out = median over the B values lam_per[0..B-1] (one wave).
__global__ void k_median_scalar(const double* lam_per, int B, double* lam_out) {
  const int lane = threadIdx.x & 63;
  const double x = lane < B ? lam_per[lane] : 0.0;
  const double med = wave_median<double>(x, B);
  if (threadIdx.x == 0) *lam_out = med;
}

template <typename R>
__global__ void k_cvt(const double* src, R* dst, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (R)src[e];
}

__global__ void k_fill_u32(unsigned* p, unsigned v, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

}  // namespace tsk
