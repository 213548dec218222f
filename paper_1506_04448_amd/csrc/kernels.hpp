// Device kernels of the sketched robust tensor power method (gfx950, wave64).
//
// Layouts (device):
//   hx  [B][3][n]  uint32  (h << 1) | (xi < 0): packed bucket and sign
//   hxs [B][3][n]  uint32  the same entries sorted by bucket (stable in i)
//   ord [B][3][n]  uint32  the index i of each sorted entry
//   spectra        cx<R>[B][b/2+1]  half spectrum of each of the B sketches
//   vectors        R[L][n]; per-sketch estimates R[L][B][n]
//   twiddles       cx<R>[twid_len(H, NT)]: per-pass table, then W_b^k (fft.hpp)
//
// Real transforms of length b use one complex transform of length H = b/2 on
// the even/odd packing z_s = x_2s + i x_2s+1, so every work-group holds only
// H complex values in LDS.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "fft.hpp"

namespace tsk {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// v from lane + o of the wave (own value past lane 63).  `lane` is passed in
// so callers can hide it from the compiler: the lane addresses are then
// recomputed per call instead of being kept live across a whole kernel.
__device__ __forceinline__ double wave_down(double v, int o, int lane) {
  const int idx = ((lane + o) < 64 ? lane + o : lane) << 2;
  const int lo = __builtin_amdgcn_ds_bpermute(idx, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(idx, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// Sum over the work-group, returned to every thread.  `red` holds NT/64
// doubles.  Each wave reduces its lanes; then every thread adds the wave sums
// in the same fixed tree order, so all threads return the same value.  The
// barrier in front keeps a previous call's readers of `red` safe.
template <int NT>
__device__ double block_sum(double v, double* red) {
  constexpr int W = NT / 64;
  int lane = threadIdx.x & 63;
  asm volatile("" : "+v"(lane));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += wave_down(v, o, lane);
  __syncthreads();
  if (lane == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r[W];
#pragma unroll
  for (int i = 0; i < W; ++i) r[i] = red[i];
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < o; ++i) r[i] += r[i + o];
  return r[0];
}

// Median of the values held by lanes 0..B-1 of a wave (B <= 64), returned to
// every lane; must be called by all 64 lanes.  Ranks break ties by lane, so
// they are a permutation; for even B the two middle values are averaged.
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

// Deterministic count sketch: the entries sharing a bucket are summed by one
// thread in increasing index order; store(bucket, sum) writes the result.
template <typename R, typename GetU, typename Store>
__device__ __forceinline__ void count_sketch(const uint32_t* __restrict__ hxs,
                                             const uint32_t* __restrict__ ord, int n, int nt,
                                             GetU getu, Store store) {
  for (int p = threadIdx.x; p < n; p += nt) {
    uint32_t e = hxs[p];
    const uint32_t bk = e >> 1;
    if (p > 0 && (hxs[p - 1] >> 1) == bk) continue;
    R acc = R(0);
    int q = p;
    while (true) {
      const R val = getu(ord[q]);
      acc += (e & 1u) ? -val : val;
      if (++q >= n) break;
      e = hxs[q];
      if ((e >> 1) != bk) break;
    }
    store(bk, acc);
  }
}

// Store of a real sequence x_t into the even/odd packing z_{t/2}.
template <typename R>
__device__ __forceinline__ void store_packed(const Soa<R>& buf, uint32_t t, R v) {
  const int q = pidx((int)(t >> 1));
  if (t & 1u) buf.im[q] = v;
  else buf.re[q] = v;
}
template <typename R>
__device__ __forceinline__ R load_packed(const Soa<R>& buf, uint32_t t) {
  const int q = pidx((int)(t >> 1));
  return (t & 1u) ? buf.im[q] : buf.re[q];
}

// X_k of a real length-b sequence from the length-H transform Z of its
// packing: X_k = (Z_k + conj Z_{H-k})/2 + W_b^k (Z_k - conj Z_{H-k})/(2i).
template <typename R>
__device__ __forceinline__ cx<R> r2c_post(cx<R> Za, cx<R> Zb, cx<R> w) {
  const cx<R> c = cconj(Zb);
  const cx<R> e = cscale(cadd(Za, c), R(0.5));
  const cx<R> d = csub(Za, c);
  const cx<R> o = {R(0.5) * d.y, R(-0.5) * d.x};
  return cadd(e, cmul(w, o));
}

// Packing for a real inverse transform: Y_k = E_k + i O_k with
// E_k = (X_k + conj X_{H-k})/2, O_k = (X_k - conj X_{H-k})/2 * conj(W_b^k).
template <typename R>
__device__ __forceinline__ cx<R> c2r_pack(cx<R> Xk, cx<R> XHk, cx<R> Wk) {
  const cx<R> c = cconj(XHk);
  const cx<R> E = cscale(cadd(Xk, c), R(0.5));
  const cx<R> O = cmulc(cscale(csub(Xk, c), R(0.5)), Wk);
  return {E.x - O.y, E.y + O.x};
}

// Both bins k and H-k of a real sequence's spectrum, twice over, from the
// half-length transform Z of its even/odd packing: with c = conj Z[H-k],
// e = Z[k] + c and o = (Z[k] - c) / i, 2 X[k] = e + W_b^k o and
// 2 X[H-k] = conj(e - W_b^k o).  Returns 2 X[k] in xk and conj(2 X[H-k]) in xm.
template <typename R>
__device__ __forceinline__ void r2c_pair2(cx<R> Zk, cx<R> Zm, cx<R> w, cx<R>& xk, cx<R>& xm) {
  const cx<R> e = {Zk.x + Zm.x, Zk.y - Zm.y};
  const cx<R> o = {Zk.y + Zm.y, Zm.x - Zk.x};
  const cx<R> t = cmul(w, o);
  xk = cadd(e, t);
  xm = csub(e, t);
}

// The packing Y of c2r_pack for both k and H-k, twice over: with
// E = X[k] + conj X[H-k] and O = (X[k] - conj X[H-k]) conj(W_b^k),
// 2 Y[k] = E + i O and 2 Y[H-k] = conj(E) + i conj(O).
template <typename R>
__device__ __forceinline__ void c2r_pair2(cx<R> Xk, cx<R> Xm, cx<R> w, cx<R>& yk, cx<R>& ym) {
  const cx<R> E = {Xk.x + Xm.x, Xk.y - Xm.y};
  const cx<R> O = cmulc(cx<R>{Xk.x - Xm.x, Xk.y + Xm.y}, w);
  yk = {E.x - O.y, E.y + O.x};
  ym = {E.x + O.y, O.x - E.y};
}

// Threads per work-group for a half-length H = 2^logh transform held in LDS:
// eight complex values per thread (radix-8 passes), 64 to 1024 threads.
template <typename R>
constexpr int threads_for_h(int logh) {
  return logh >= 13 ? 1024 : (logh >= 9 ? (1 << (logh - 3)) : 64);
}

// ---------------------------------------------------------------------------
// Threads of a power-step work-group.  FP32 holds 16 points per thread
// (radix-16 passes) from H = 1024 on, so that at b = 16384 a work-group needs
// about 76 KB of LDS and 128 VGPRs and two of them share a CU; FP64 holds 8
// points per thread (radix 8), one work-group per CU at that size.
// ---------------------------------------------------------------------------
template <typename R>
constexpr int power_threads(int logh) {
  return (sizeof(R) == 4 && logh >= 10) ? (1 << (logh - 4)) : threads_for_h<R>(logh);
}
// Waves per SIMD the power kernel is compiled for: two FP32 work-groups per
// CU while the sequence takes at most half the LDS (H <= 8192), one otherwise.
template <typename R>
constexpr int power_waves(int logh) {
  return power_threads<R>(logh) / ((sizeof(R) == 4 && logh <= 13) ? 128 : 256) < 1
             ? 1
             : power_threads<R>(logh) / ((sizeof(R) == 4 && logh <= 13) ? 128 : 256);
}

constexpr size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Dynamic LDS of one power-step work-group, in bytes:
//   [0, 128)          reduction scratch (16 doubles)
//   [128, off_u)      the padded half-length sequence, split re/im (also the
//                     staging area of the median prologue)
//   [off_u, off_tab)  the vector u (n values)
//   [off_tab, end)    when `tab`: the table rows read by the count sketches of
//                     modes 2 and 3 (sorted buckets, indices) and by the
//                     read-off (mode 1), five rows of n words.
template <typename R>
constexpr size_t power_lds_off_u(int logh) {
  return align16(128 + sizeof(R) * 2 * (size_t)padded_len(1 << logh));
}
template <typename R>
constexpr size_t power_lds_off_tab(int logh, int n) {
  return power_lds_off_u<R>(logh) + align16(sizeof(R) * (size_t)n);
}
template <typename R>
constexpr size_t power_lds_bytes(int logh, int n, bool tab) {
  return power_lds_off_tab<R>(logh, n) + (tab ? (size_t)20 * n : 0);
}

// Zero `bytes` bytes of LDS from a 16-byte aligned start, 16 bytes per store.
template <int NT>
__device__ __forceinline__ void zero_lds(void* p, int bytes) {
  float4* q = reinterpret_cast<float4*>(p);
  const int n16 = bytes >> 4;
  for (int t = threadIdx.x; t < n16; t += NT) q[t] = make_float4(0.f, 0.f, 0.f, 0.f);
  float* tail = reinterpret_cast<float*>(q + n16);
  const int nt = (bytes & 15) >> 2;
  if ((int)threadIdx.x < nt) tail[threadIdx.x] = 0.f;
}

// Copy `count` consecutive values from global memory to LDS, U loads in
// flight per thread before the first store.
template <int NT, int U, typename T>
__device__ __forceinline__ void copy_to_lds(T* dst, const T* __restrict__ src, int count) {
  for (int base = 0; base < count; base += NT * U) {
    T v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = base + q * NT + (int)threadIdx.x;
      if (e < count) v[q] = src[e];
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int e = base + q * NT + (int)threadIdx.x;
      if (e < count) dst[e] = v[q];
    }
  }
}

// Coordinates per chunk of the median prologue: B staged rows plus the two
// selected order statistics must fit `cap` LDS values.
__device__ __forceinline__ int median_chunk(int n, int B, int cap) {
  const int c = cap / (B + 2);
  return n < c ? n : c;
}

// Sorts v[0..N) ascending in registers with Batcher's odd-even merge network
// (63 compare-exchanges for N = 16); N a power of two, all indices fixed at
// compile time.
template <int N, typename R>
__device__ __forceinline__ void sort_network(R (&v)[N]) {
#pragma unroll
  for (int p = 1; p < N; p <<= 1)
#pragma unroll
    for (int k = p; k >= 1; k >>= 1)
#pragma unroll
      for (int j = k % p; j + k < N; j += 2 * k)
#pragma unroll
        for (int i = 0; i < k && i + j + k < N; ++i)
          if ((i + j) / (2 * p) == (i + j + k) / (2 * p)) {
            const R lo = fmin(v[i + j], v[i + j + k]), hi = fmax(v[i + j], v[i + j + k]);
            v[i + j] = lo;
            v[i + j + k] = hi;
          }
}

// Median of B <= N values get(0..B-1) by the network in registers (padded
// with +inf): the element of rank (B-1)/2, or for even B the mean of ranks
// B/2-1 and B/2; any NaN among them gives NaN.
template <int N, typename R, typename Get>
__device__ __forceinline__ R network_median(Get get, int B) {
  R v[N];
  bool nan = false;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    v[j] = j < B ? get(j) : R(__builtin_inf());
    nan |= __builtin_isnan(v[j]);
  }
  sort_network(v);
  const int ra = (B - 1) / 2, rb = B / 2;
  R xa = v[0], xc = v[0];
#pragma unroll
  for (int j = 1; j < N; ++j) {
    xa = j == ra ? v[j] : xa;
    xc = j == rb ? v[j] : xc;
  }
  const R med = (B & 1) ? xa : (xa + xc) * R(0.5);
  return nan ? R(__builtin_nan("")) : med;
}

// ---------------------------------------------------------------------------
// Median prologue: u = vbar / ||vbar||, vbar_i = med_m Vprev[tau][m][i], for
// the n coordinates of one restart, into u[] (LDS or global).  Falls back to
// Uprev[tau] when ||vbar|| is zero or not finite.  The median is the element
// of rank (B-1)/2 (odd B) or the mean of ranks B/2-1 and B/2 (even B), ranks
// breaking ties by sketch index; any NaN among the B values gives NaN.  For
// B <= 16 each thread sorts one coordinate's values with a network in
// registers; otherwise every (coordinate, sketch) pair ranks its value in
// parallel and the two selected ranks are written to LDS.  `stage` is LDS
// scratch of `cap` values; with
// `staged` the whole B x n block (one chunk) is already there, row m at m*n.
// Returns true when the median vector was usable.
// ---------------------------------------------------------------------------
template <typename R, int NT>
__device__ __forceinline__ bool median_prologue(const R* __restrict__ Vprev, const R* __restrict__ Uprev, int tau,
                                                int n, int B, R* u, R* stage, int cap, double* red, bool staged) {
  const R* vb = Vprev + (size_t)tau * B * n;
  const int CH = median_chunk(n, B, cap);
  R* selA = stage + B * CH;
  R* selC = selA + CH;
  const int ra = (B - 1) / 2, rb = B / 2;
  double ss = 0.0;
  for (int c0 = 0; c0 < n; c0 += CH) {
    const int cw = min(CH, n - c0);
    if (!staged) {
      __syncthreads();  // the previous chunk's readers are done
      for (int e = threadIdx.x; e < B * cw; e += NT) {
        const int mm = e / cw, ii = e - mm * cw;
        stage[mm * CH + ii] = vb[(size_t)mm * n + c0 + ii];
      }
      __syncthreads();
    }
    if (B <= 16) {
      // One coordinate per thread: its B values (padded with +inf) sorted by
      // a network in registers; the order statistics are the same values the
      // ranking below selects.
      for (int ii = threadIdx.x; ii < cw; ii += NT) {
        const R med = network_median<16, R>([&](int j) { return stage[j * CH + ii]; }, B);
        u[c0 + ii] = med;
        ss += (double)med * (double)med;
      }
      continue;
    }
    for (int e = threadIdx.x; e < B * cw; e += NT) {
      const int mm = e / cw, ii = e - mm * cw;
      const R x = stage[mm * CH + ii];
      int r = 0;
      for (int j = 0; j < B; ++j) {
        const R o = stage[j * CH + ii];
        r += (o < x) || (o == x && j < mm);
      }
      if (r == ra) selA[ii] = x;
      if (r == rb) selC[ii] = x;
    }
    __syncthreads();
    for (int ii = threadIdx.x; ii < cw; ii += NT) {
      bool nan = false;
      for (int j = 0; j < B; ++j) nan |= __builtin_isnan(stage[j * CH + ii]);
      R med = (B & 1) ? selA[ii] : (selA[ii] + selC[ii]) * R(0.5);
      if (nan) med = R(__builtin_nan(""));
      u[c0 + ii] = med;
      ss += (double)med * (double)med;
    }
  }
  const double nrm = sqrt(block_sum<NT>(ss, red));
  const bool ok = nrm > 0.0 && nrm < __builtin_inf();
  if (ok) {
    const R inv = R(1.0 / nrm);
    for (int i = threadIdx.x; i < n; i += NT) u[i] *= inv;
  } else {
    const R* up = Uprev + (size_t)tau * n;
    for (int i = threadIdx.x; i < n; i += NT) u[i] = up[i];
  }
  __syncthreads();
  return ok;
}

// ---------------------------------------------------------------------------
// Power step / evaluation: one work-group per (sketch m, restart tau).
//   u     = Uprev[tau] (PRE false) or the normalised median of Vprev[tau] (PRE)
//   A_k   = S_k conj(F(s2 u)_k);   P_k = A_k conj(F(s3 u)_k)
//   sbar  = F^-1(P);  v_i = xi1(i) sbar[h1(i)]  -> V[tau][m]
//   mode 1 also writes lam_per[tau][m] = u . v.
// With the modes permuted (rd, sa, sb) the same read-off is the derivative of
// <s, s_1(u) * s_2(u) * s_3(u)> along mode rd.
// ---------------------------------------------------------------------------
template <typename R>
struct PowerArgs {
  const uint32_t* hx;
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B;
  const cx<R>* S;       // [B][H+1]
  const cx<R>* twg;     // [twid_len(H, NT)]
  const R* Uprev;       // [L][n]
  const R* Uy;          // [L][n] or null: the second count sketch's vector (two-vector
                        // contraction; not with PRE or mode 1)
  const R* Vprev;       // [L][B][n]   (PRE)
  R* Ucur;              // [L][n]      (PRE, written by m == 0)
  int32_t* flags;       // [L]         (PRE, nullable)
  R* V;                 // [L][B][n]
  double* lam_per;      // [L][B]      (mode 1)
  int tau0;
  int prefix;           // median prologue (selects the PRE instantiation)
  int mode;
  int tab_lds;          // table rows staged in LDS (power_lds_bytes with tab)
  int rd, sa, sb;       // table modes of the read-off and of the two count sketches
                        // (0, 1, 2 for Proposition 1; permuted for gradients)
};

// PRE selects the median prologue (u from Vprev) at compile time; the two
// variants show up as separate kernels in traces.
template <typename R, int LOGB, bool PRE>
__global__ __launch_bounds__(power_threads<R>(LOGB - 1), power_waves<R>(LOGB - 1)) void k_power(PowerArgs<R> a) {
  constexpr int LOGH = LOGB - 1;
  constexpr int NT = power_threads<R>(LOGH);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  constexpr int PL = padded_len(H);
  // Thread tid owns the pairs (k, H-k) for k = tid + q NT < H/2; thread 0
  // also owns k = H/2, which pairs with itself.
  constexpr int PK = (H / 2 + NT - 1) / NT;
  constexpr bool FULL = (H / 2) % NT == 0;
  // With a last pass of radix 2, the forward transforms stop before it and
  // the spectral products form X[k], X[H-k] from its inputs; the inverse stops
  // before it and the read-off forms just the outputs it reads.
  constexpr bool FUSE = fft_last_radix(H, NT) == 2 && H >= 64;
  constexpr int TLAST = pass_table_len(H, NT) - H / 2;  // W_H^j, j < H/2, in the pass table
  extern __shared__ __align__(16) unsigned char lds[];
  const int n = a.n;
  const int B = a.B;
  double* red = reinterpret_cast<double*>(lds);
  R* re = reinterpret_cast<R*>(lds + 128);
  R* im = re + PL;
  R* u = reinterpret_cast<R*>(lds + power_lds_off_u<R>(LOGH));
  uint32_t* stab = reinterpret_cast<uint32_t*>(lds + power_lds_off_tab<R>(LOGH, n));
  const Soa<R> buf{re, im};

  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const int tau = a.tau0 + blockIdx.y;
  const size_t tb = (size_t)m * 3 * n;
  const cx<R>* Sm = a.S + (size_t)m * (H + 1);
  const cx<R>* wkg = a.twg + pass_table_len(H, NT);
  const bool tab_lds = a.tab_lds != 0;

  // Global loads in the order they are needed: the table rows and u, or the
  // previous step's estimates for the median prologue, first.
  for (int e = tid; e < n; e += NT) {
    uint32_t t0 = 0, t1 = 0, t2 = 0, t3 = 0, t4 = 0;
    R uu = R(0);
    if (tab_lds) {
      t0 = a.hxs[tb + (size_t)a.sa * n + e];
      t1 = a.ord[tb + (size_t)a.sa * n + e];
      t2 = a.hxs[tb + (size_t)a.sb * n + e];
      t3 = a.ord[tb + (size_t)a.sb * n + e];
      t4 = a.hx[tb + (size_t)a.rd * n + e];
    }
    if (!PRE) uu = a.Uprev[(size_t)tau * n + e];
    if (tab_lds) {
      stab[e] = t0;
      stab[n + e] = t1;
      stab[2 * n + e] = t2;
      stab[3 * n + e] = t3;
      stab[4 * n + e] = t4;
    }
    if (!PRE) u[e] = uu;
  }
  const bool staged = PRE && median_chunk(n, B, 2 * PL) == n;
  if (staged) copy_to_lds<NT, 4>(re, a.Vprev + (size_t)tau * B * n, B * n);
  // Then this sketch's spectrum values owned by the thread (they become the
  // running products p0/p1) and the twiddles W_b^tid and W_b^(q NT)
  // (uniform); issued after the loads above, they stay in flight through the
  // prologue and the first count sketch (loads complete in issue order, so
  // waiting for the earlier ones does not wait for these).  W_b^k for
  // k = tid + q NT is formed as W_b^tid W_b^(q NT) when needed (two registers
  // instead of 2 PK), W_b^(H-k) = -conj(W_b^k) and W_b^(H/2) = -i.
  cx<R> p0[PK], p1[PK], pmid;
  cx<R> wq[PK];
#pragma unroll
  for (int q = 0; q < PK; ++q) {
    const int k = tid + q * NT;
    wq[q] = wkg[q * NT];
    if (!FULL && k >= H / 2) break;
    p0[q] = Sm[k];
    p1[q] = Sm[H - k];
  }
  const cx<R> wt = wkg[tid < H / 2 ? tid : 0];
  auto wk = [&](int q) -> cx<R> { return q == 0 ? wt : cmul(wt, wq[q]); };
  if (tid == 0) pmid = Sm[H / 2];
  const Twid<R> tw{a.twg, wkg};
  __syncthreads();  // staged tables, u or the estimates visible

  if constexpr (PRE) {
    const bool ok = median_prologue<R, NT>(a.Vprev, a.Uprev, tau, n, B, u, re, 2 * PL, red, staged);
    if (m == 0) {
      for (int i = tid; i < n; i += NT) a.Ucur[(size_t)tau * n + i] = u[i];
      if (tid == 0 && !ok && a.flags) a.flags[tau] |= 1;
    }
  }

  auto getu = [&](uint32_t i) -> R { return u[i]; };
  auto store = [&](uint32_t t, R v) { store_packed(buf, t, v); };
#pragma unroll 1
  for (int mode_j = 1; mode_j <= 2; ++mode_j) {
    if (!PRE && a.Uy && mode_j == 2) {
      // two-vector contraction: the second count sketch takes y (u is not
      // read again: mode 0 has no lambda read-off)
      int oe = threadIdx.x, ot2 = tau;
      asm volatile("" : "+v"(oe), "+s"(ot2));
      for (int e = oe; e < n; e += NT) u[e] = a.Uy[(size_t)ot2 * n + e];
    }
    zero_lds<NT>(re, 2 * PL * (int)sizeof(R));
    __syncthreads();
    if (tab_lds)
      count_sketch<R>(stab + (mode_j - 1) * 2 * n, stab + (mode_j - 1) * 2 * n + n, n, NT, getu, store);
    else
      count_sketch<R>(a.hxs + tb + (size_t)(mode_j == 1 ? a.sa : a.sb) * n,
                      a.ord + tb + (size_t)(mode_j == 1 ? a.sa : a.sb) * n, n, NT, getu, store);
    __syncthreads();
    fft_soa<R, LOGH, NT, false, false, FUSE>(buf, tw);
    // Opaque thread index: the pair indices are recomputed here rather than
    // kept live (or spilled) from the loads at the start.
    int ot = threadIdx.x;
    asm volatile("" : "+v"(ot));
    // Bins k and H-k need Z[k] and Z[H-k]; fused, Z[k] comes from the inputs
    // k, k + H/2 of the skipped pass and Z[H-k] from j, j + H/2, j = H/2 - k.
    constexpr int M = FUSE ? H / 2 : H;
    const int P0 = pidx(ot), Pm = pidx(NT - ot);
#pragma unroll
    for (int q = 0; q < PK; ++q) {
      const int k = ot + q * NT;
      if (!FULL && k >= H / 2) break;
      cx<R> w0 = wk(q);
      asm volatile("" : "+v"(w0.x), "+v"(w0.y));  // formed here, not hoisted out of the mode loop
      // padded positions of k and of its mirror M - k (0 for k = 0)
      const int pk = FULL ? P0 + poff(q * NT) : pidx(k);
      int pm = FULL ? Pm + poff(M - NT - q * NT) : pidx((M - k) & (M - 1));
      if (FULL && q == 0) pm = ot == 0 ? 0 : pm;
      cx<R> Za, Zb;
      if constexpr (FUSE) {
        const cx<R> wH = cmul(w0, w0);  // W_H^k = (W_b^k)^2; W_H^(H/2-k) = -conj(W_H^k)
        Za = cadd(buf.at(pk), cmul(wH, buf.at(pk + poff(H / 2))));
        const cx<R> Zc = cadd(buf.at(pm), cmulc(buf.at(pm + poff(H / 2)), wH));
        Zb = (q == 0 && k == 0) ? Za : Zc;  // X[H] is X[0]
      } else {
        Za = buf.at(pk);
        Zb = buf.at(pm);
      }
      cx<R> xk, xm;
      r2c_pair2(Za, Zb, w0, xk, xm);
      p0[q] = cmulc(p0[q], xk);  // P[k] conj(2 X[k])
      p1[q] = cmul(p1[q], xm);   // P[H-k] conj(2 X[H-k])
      // this pair finished before the next pair's loads
      asm volatile("" : "+v"(p0[q].x), "+v"(p0[q].y), "+v"(p1[q].x), "+v"(p1[q].y) : : "memory");
    }
    if (tid == 0) {  // bin H/2: 2 X[H/2] = 2 conj(Z[H/2])
      const cx<R> Z = FUSE ? csub(buf.get(0), buf.get(H / 2)) : buf.get(H / 2);
      pmid = cscale(cmul(pmid, Z), R(2));
    }
    __syncthreads();
  }
  // Half-length packing of the real inverse transform of P (twice over).
  int ot = threadIdx.x;
  asm volatile("" : "+v"(ot));
  const int P0 = pidx(ot), Pm = pidx(NT - ot);
#pragma unroll
  for (int q = 0; q < PK; ++q) {
    const int k = ot + q * NT;
    if (!FULL && k >= H / 2) break;
    const cx<R> w0 = wk(q);
    cx<R> yk, ym;
    c2r_pair2(p0[q], p1[q], w0, yk, ym);
    buf.put_at(FULL ? P0 + poff(q * NT) : pidx(k), yk);
    if (k > 0) buf.put_at(FULL ? Pm + poff(H - NT - q * NT) : pidx(H - k), ym);
  }
  if (tid == 0) buf.put(H / 2, cscale(cconj(pmid), R(2)));
  __syncthreads();
  // For n small against H the inverse also leaves out the pass before the
  // last (radix R3, stride NS3).  Its inputs are the NS3-point transforms D_g
  // of the subsequences g + 2 R3 t (g < 2 R3, D_g at g NS3 + k), so each
  // output the read-off needs is z[p] = sum_g W_H^{-g p} D_g[p mod NS3]:
  // 2 R3 terms per output instead of the whole pass.
  constexpr int RMX = fft_rmax(H, NT);
  constexpr bool PRUNABLE = FUSE && passes_from(H, 1, RMX) >= 3;
  constexpr int NS3 = pass_stride(H, NT, 1);
  constexpr int R3 = pass_radix(H, NS3, RMX);
  const bool prune = PRUNABLE && n * R3 <= H;
  if constexpr (PRUNABLE) {
    fft_soa<R, LOGH, NT, true, false, 2>(buf, tw);
    if (!prune) fft_soa_from<R, LOGH, NT, true, NS3, 1>(buf, tw);
  } else {
    fft_soa<R, LOGH, NT, true, false, FUSE>(buf, tw);
  }

  // Each forward product carried a factor 2 and the packing another.
  const R scale = R(1) / R(4 * b);
  // Read-off addresses formed here from opaque copies of the indices, so the
  // compiler does not keep them live (or spill them) through the transforms.
  int om = m, otau = tau, orid = tid;
  asm volatile("" : "+v"(orid), "+s"(om), "+s"(otau));
  const uint32_t* hx1 = a.hx + (size_t)om * 3 * n + (size_t)a.rd * n;
  R* Vrow = a.V + ((size_t)otau * B + om) * n;
  double acc = 0.0;
  for (int i = orid; i < n; i += NT) {
    const uint32_t e = tab_lds ? stab[4 * n + i] : hx1[i];
    R val;
    if constexpr (FUSE) {  // the skipped last inverse pass(es), for this output only
      const uint32_t t = e >> 1, p = t >> 1;
      const int j = (int)(p & (uint32_t)(H / 2 - 1));
      const cx<R> W = a.twg[TLAST + j];  // W_H^j; W_H^{-p} = +-conj(W)
      cx<R> E0, E1;
      if (PRUNABLE && prune) {
        // E_c = sum_r (W_H^{-2p})^r D_{c+2r}[k], two-level Horner (groups of
        // RI terms), so no term passes through more than a few roundings.
        constexpr int RI = R3 >= 4 ? 4 : R3;
        const int k = (int)(p & (uint32_t)(NS3 - 1));
        const int pk = pidx(k);
        auto d = [&](int g) -> cx<R> {
          return buf.at(NS3 % 64 == 0 ? pk + poff(g * NS3) : pidx(g * NS3 + k));
        };
        auto mad = [](cx<R> x, cx<R> w, cx<R> y) -> cx<R> {
          return {x.x * w.x - x.y * w.y + y.x, x.x * w.y + x.y * w.x + y.y};
        };
        const cx<R> w2 = cconj(cmul(W, W));
        cx<R> wo = w2;
#pragma unroll
        for (int s2 = 1; s2 < RI; s2 *= 2) wo = cmul(wo, wo);
        cx<R> E[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          cx<R> acc{R(0), R(0)};
#pragma unroll
          for (int r1 = R3 / RI - 1; r1 >= 0; --r1) {
            cx<R> in = d(c + 2 * (r1 * RI + RI - 1));
#pragma unroll
            for (int r0 = RI - 2; r0 >= 0; --r0) in = mad(in, w2, d(c + 2 * (r1 * RI + r0)));
            acc = r1 == R3 / RI - 1 ? in : mad(acc, wo, in);
          }
          E[c] = acc;
        }
        E0 = E[0];
        E1 = E[1];
      } else {
        E0 = buf.get(j);
        E1 = buf.get(j + H / 2);
      }
      const cx<R> c = cmulc(E1, W);
      const cx<R> X = p < (uint32_t)(H / 2) ? cadd(E0, c) : csub(E0, c);
      val = ((t & 1u) ? X.y : X.x) * scale;
    } else {
      val = load_packed(buf, e >> 1) * scale;
    }
    const R v = (e & 1u) ? -val : val;
    Vrow[i] = v;
    acc += (double)u[i] * (double)v;
  }
  if (a.mode == 1) {
    const double lam = block_sum<NT>(acc, red);
    if (tid == 0) a.lam_per[(size_t)tau * B + m] = lam;
  }
}

// Threads of the median kernel: the 64-value network holds 64 values per
// thread in registers (FP64: 128 VGPRs, so one wave per SIMD).
template <typename R>
constexpr int median_threads() { return sizeof(R) == 8 ? 256 : 512; }

// u_out[tau] = normalised median of V[tau] (fallback u_in, flag), grid = L,
// median_threads<R>() threads.  For B <= 64 each thread takes whole coordinates: its B values
// straight from global memory (coalesced across threads for each m) into a
// sorting network; larger B goes through the ranking prologue.
template <typename R>
__global__ __launch_bounds__(median_threads<R>()) void k_median_norm(const R* V, const R* Uin, R* Uout,
                                                                     int32_t* flags, int n, int B) {
  constexpr int NT = median_threads<R>();
  __shared__ __align__(16) R stage[4096];
  __shared__ double red[NT / 64];
  const int tau = blockIdx.x;
  R* u = Uout + (size_t)tau * n;  // written in place, then normalised
  bool ok;
  if (B <= 64) {
    const R* Vt = V + (size_t)tau * B * n;
    double ss = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
      auto get = [&](int j) { return Vt[(size_t)j * n + i]; };
      const R med = B <= 16   ? network_median<16, R>(get, B)
                    : B <= 32 ? network_median<32, R>(get, B)
                              : network_median<64, R>(get, B);
      u[i] = med;
      ss += (double)med * (double)med;
    }
    const double nrm = sqrt(block_sum<NT>(ss, red));
    ok = nrm > 0.0 && nrm < __builtin_inf();
    const R inv = ok ? R(1.0 / nrm) : R(0);
    const R* up = Uin + (size_t)tau * n;
    for (int i = threadIdx.x; i < n; i += NT) u[i] = ok ? u[i] * inv : up[i];  // own coordinates
  } else {
    ok = median_prologue<R, NT>(V, Uin, tau, n, B, u, stage, 4096, red, false);
  }
  if (threadIdx.x == 0 && !ok && flags) flags[tau] |= 1;
}

// ---------------------------------------------------------------------------
// Fast ALS (Appendix C, Algorithm 2): the update of one factor from the
// median estimates Vbar[r] of T(I, x_r, y_r) and the other two factors X, Y
// (rows r = 0..k-1):  A = G^+ Vbar,  G = (X X^T) o (Y Y^T),  lambda_r = ||A_r||,
// A_r /= lambda_r.

// Vbar[r][i] = med_m V[r][m][i] (no normalisation), FP64 out; grid = k rows,
// median_threads<R>() threads.  B <= 64 by sorting networks, else by ranks.
template <typename R>
__global__ __launch_bounds__(median_threads<R>()) void k_median_rows(const R* V, double* Vbar, int n, int B) {
  constexpr int NT = median_threads<R>();
  const int r = blockIdx.x;
  const R* Vr = V + (size_t)r * B * n;
  for (int i = threadIdx.x; i < n; i += NT) {
    auto get = [&](int j) { return Vr[(size_t)j * n + i]; };
    R med;
    if (B <= 16) {
      med = network_median<16, R>(get, B);
    } else if (B <= 32) {
      med = network_median<32, R>(get, B);
    } else if (B <= 64) {
      med = network_median<64, R>(get, B);
    } else {
      const int ra = (B - 1) / 2, rb = B / 2;
      R xa = R(0), xc = R(0);
      bool nan = false;
      for (int mm = 0; mm < B; ++mm) {
        const R x = get(mm);
        nan |= __builtin_isnan(x);
        int rank = 0;
        for (int j = 0; j < B; ++j) {
          const R o = get(j);
          rank += (o < x) || (o == x && j < mm);
        }
        if (rank == ra) xa = x;
        if (rank == rb) xc = x;
      }
      med = nan ? R(__builtin_nan("")) : ((B & 1) ? xa : (xa + xc) * R(0.5));
    }
    Vbar[(size_t)r * n + i] = (double)med;
  }
}

// G[r][s] = (x_r . x_s)(y_r . y_s), FP64; grid = (k, k), 256 threads; fixed
// reduction order, so G is exactly symmetric.
__global__ __launch_bounds__(256) void k_als_gram(const double* X, const double* Y, double* G, int n, int k) {
  __shared__ double red[4];
  const int r = blockIdx.x, c = blockIdx.y;
  const int lo = min(r, c), hi = max(r, c);
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    sx += X[(size_t)lo * n + i] * X[(size_t)hi * n + i];
    sy += Y[(size_t)lo * n + i] * Y[(size_t)hi * n + i];
  }
  const double gx = block_sum<256>(sx, red);
  const double gy = block_sum<256>(sy, red);
  if (threadIdx.x == 0) G[(size_t)r * k + c] = gx * gy;
}

// Jacobi sweeps on the symmetric k x k matrix A (k <= 128, row-major in
// LDS), accumulating the rotations into E (LDS, the identity on entry), by
// the 256 threads of a work-group: the round-robin order, every round
// rotating k/2 disjoint index pairs at once (player 0 fixed, the others
// moving round a circle; a dummy player when k is odd), until the
// off-diagonal mass is below 1e-30 of the total (at most 60 sweeps).  On
// return A is diagonal to that accuracy: A = E diag E^T of the input.
__device__ inline void jacobi_sweeps(double* A, double* E, int k, double* red) {
  __shared__ double rc[64], rs[64];
  __shared__ int rp[64], rq[64];
  const int tid = threadIdx.x;
  const int m = k + (k & 1);  // players
  const int np = m / 2;       // pairs per round
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < k * k; e += 256) {
      const double v = A[e] * A[e];
      tot += v;
      if (e / k != e % k) off += v;
    }
    off = block_sum<256>(off, red);
    tot = block_sum<256>(tot, red);
    if (!(off > 1e-30 * tot)) break;  // uniform: every thread has the same sums
    for (int round = 0; round + 1 < m; ++round) {
      if (tid < np) {
        const int a = tid == 0 ? 0 : (round + tid) % (m - 1) + 1;
        const int b = tid == 0 ? round % (m - 1) + 1 : (round - tid + m - 1) % (m - 1) + 1;
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        if (q < k) {
          const double apq = A[p * k + q];
          if (apq != 0.0) {
            const double theta = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        rp[tid] = p;
        rq[tid] = q;
        rc[tid] = c;
        rs[tid] = s;
      }
      __syncthreads();
      // A <- J^T A J over the 2 x 2 blocks (rows of pair i, columns of pair
      // j), every block at once: the column rotation of pair j, then the row
      // rotation of pair i on its result; E <- E J.  One pass, so a round
      // takes two barriers.
      for (int e = tid; e < np * np; e += 256) {
        const int i = e / np, j = e - i * np;
        const double si = rs[i], sj = rs[j];
        if (si == 0.0 && sj == 0.0) continue;
        const int p = rp[i], q = rq[i], u = rp[j], v = rq[j];
        const bool qi = q < k, vj = v < k;  // a dummy player has no row / column
        double apu = A[p * k + u], apv = vj ? A[p * k + v] : 0.0;
        double aqu = qi ? A[q * k + u] : 0.0, aqv = (qi && vj) ? A[q * k + v] : 0.0;
        if (sj != 0.0) {
          const double cj = rc[j];
          const double tpu = cj * apu - sj * apv, tpv = sj * apu + cj * apv;
          const double tqu = cj * aqu - sj * aqv, tqv = sj * aqu + cj * aqv;
          apu = tpu;
          apv = tpv;
          aqu = tqu;
          aqv = tqv;
        }
        if (si != 0.0) {
          const double ci = rc[i];
          const double npu = ci * apu - si * aqu, nqu = si * apu + ci * aqu;
          const double npv = ci * apv - si * aqv, nqv = si * apv + ci * aqv;
          apu = npu;
          aqu = nqu;
          apv = npv;
          aqv = nqv;
        }
        A[p * k + u] = apu;
        if (vj) A[p * k + v] = apv;
        if (qi) A[q * k + u] = aqu;
        if (qi && vj) A[q * k + v] = aqv;
      }
      for (int e = tid; e < np * k; e += 256) {
        const int j = e / k, r = e - j * k;
        const double s = rs[j];
        if (s != 0.0) {
          const double c = rc[j];
          const int p = rp[j], q = rq[j];
          const double ep = E[r * k + p], eq = E[r * k + q];
          E[r * k + p] = c * ep - s * eq;
          E[r * k + q] = s * ep + c * eq;
        }
      }
      __syncthreads();
    }
  }
}

// P = G^+ for a symmetric k x k G (k <= 64), one work-group of 256 threads:
// Jacobi sweeps to G = E diag(d) E^T, then P = E diag(1/d) E^T over the
// eigenvalues d > 1e-12 max|d| (the others dropped).
__global__ __launch_bounds__(256) void k_als_pinv(const double* G, double* P, int k) {
  __shared__ double A[64 * 64];
  __shared__ double E[64 * 64];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (int e = tid; e < k * k; e += 256) {
    A[e] = G[e];
    E[e] = (e / k == e % k) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_sweeps(A, E, k, red);
  double dmax = 0.0;
  for (int j = 0; j < k; ++j) dmax = fmax(dmax, fabs(A[j * k + j]));
  for (int e = tid; e < k * k; e += 256) {
    const int r = e / k, c = e % k;
    double acc = 0.0;
    for (int j = 0; j < k; ++j) {
      const double d = A[j * k + j];
      if (fabs(d) > 1e-12 * dmax) acc += E[r * k + j] * E[c * k + j] / d;
    }
    P[e] = acc;
  }
}

// A[r][i] = sum_s P[r][s] Vbar[s][i]; grid = (ceil(n / 256), k).
__global__ __launch_bounds__(256) void k_als_apply(const double* P, const double* Vbar, double* A, int n, int k) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= n) return;
  double acc = 0.0;
  for (int s2 = 0; s2 < k; ++s2) acc += P[(size_t)r * k + s2] * Vbar[(size_t)s2 * n + i];
  A[(size_t)r * n + i] = acc;
}

// lambda_r = ||A_r||, A_r /= lambda_r (rows of zero norm stay), and the
// factor in the power kernel's precision; grid = k, 256 threads.
template <typename R>
__global__ __launch_bounds__(256) void k_als_normalize(double* A, R* Ar, double* lam, int n) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  double* row = A + (size_t)r * n;
  double ss = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) ss += row[i] * row[i];
  const double nrm = sqrt(block_sum<256>(ss, red));
  const double inv = nrm > 0.0 ? 1.0 / nrm : 1.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double v = row[i] * inv;
    row[i] = v;
    Ar[(size_t)r * n + i] = (R)v;
  }
  if (threadIdx.x == 0) lam[r] = nrm;
}

// lam_med[tau] = med_m lam_per[tau][m]; one wave per restart.
__global__ void k_lam_median(const double* lam_per, double* lam_med, int L, int B) {
  const int tau = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (tau >= L) return;  // whole waves exit together
  const int lane = wave_lane();
  const double x = lane < B ? lam_per[(size_t)tau * B + lane] : 0.0;
  const double med = wave_median<double>(x, B);
  if (lane == 0) lam_med[tau] = med;
}

// ---------------------------------------------------------------------------
// FP64 rank-1 spectra, one work-group per (m, r):
//   prod[r][m] = F(s1 u_r) o F(s2 u_r) o F(s3 u_r),
//   lam_per[r][m] = <s^(m), s^(m)(u_r^(x)3)> (Parseval) when S64 is given.
// ---------------------------------------------------------------------------
struct Rank1Args {
  const uint32_t* hx;
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B;
  const double* U;          // [c][n]
  const cx<double>* twg;    // [twid_len(H, NT)]
  cx<double>* prod;         // [c][B][b/2+1]
  const cx<double>* S64;    // nullable: [B][b/2+1]
  double* lam_per;          // [c][B] when S64 != null
};

template <int LOGB>
__global__ __launch_bounds__(threads_for_h<double>(LOGB - 1)) void k_rank1(Rank1Args a) {
  constexpr int LOGH = LOGB - 1;
  constexpr int NT = threads_for_h<double>(LOGH);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  constexpr int PL = padded_len(H);
  constexpr int PK = (H / 2 + NT - 1) / NT;
  constexpr bool FULL = (H / 2) % NT == 0;
  __shared__ __align__(16) double re[2 * PL];
  __shared__ double red[16];
  double* im = re + PL;
  const Soa<double> buf{re, im};
  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const int r = blockIdx.y;
  const int n = a.n;
  const double* u = a.U + (size_t)r * n;
  const Twid<double> tw{a.twg, a.twg + pass_table_len(H, NT)};
  cx<double> p0[PK], p1[PK], pmid;
  auto getu = [&](uint32_t i) -> double { return u[i]; };
  auto store = [&](uint32_t t, double v) { store_packed(buf, t, v); };
#pragma unroll 1
  for (int j = 0; j < 3; ++j) {
    const size_t tb = ((size_t)m * 3 + j) * n;
    for (int t = tid; t < PL; t += NT) {
      re[t] = 0.0;
      im[t] = 0.0;
    }
    __syncthreads();
    count_sketch<double>(a.hxs + tb, a.ord + tb, n, NT, getu, store);
    __syncthreads();
    fft_soa<double, LOGH, NT, false>(buf, tw);
#pragma unroll
    for (int q = 0; q < PK; ++q) {
      const int k = tid + q * NT;
      if (!FULL && k >= H / 2) break;
      const cx<double> Za = buf.get(k);
      const cx<double> Zb = buf.get((H - k) & (H - 1));
      const cx<double> Xk = r2c_post(Za, Zb, tw.w(k));
      const cx<double> XHk = r2c_post(Zb, Za, tw.w(H - k));
      p0[q] = j == 0 ? Xk : cmul(p0[q], Xk);
      p1[q] = j == 0 ? XHk : cmul(p1[q], XHk);
    }
    if (tid == 0) {
      const cx<double> Z = buf.get(H / 2);
      const cx<double> X = r2c_post(Z, Z, tw.w(H / 2));
      pmid = j == 0 ? X : cmul(pmid, X);
    }
    __syncthreads();
  }
  cx<double>* P = a.prod + ((size_t)r * a.B + m) * (H + 1);
  double acc = 0.0;
  const cx<double>* S = a.S64 ? a.S64 + (size_t)m * (H + 1) : nullptr;
  // Parseval on the half spectrum: weight 1 at k = 0 and k = H, 2 elsewhere.
#pragma unroll
  for (int q = 0; q < PK; ++q) {
    const int k = tid + q * NT;
    if (!FULL && k >= H / 2) break;
    const double w = k == 0 ? 1.0 : 2.0;
    P[k] = p0[q];
    P[H - k] = p1[q];
    if (S) {
      const cx<double> s0 = S[k], s1 = S[H - k];
      acc += w * ((s0.x * p0[q].x + s0.y * p0[q].y) + (s1.x * p1[q].x + s1.y * p1[q].y));
    }
  }
  if (tid == 0) {
    P[H / 2] = pmid;
    if (S) acc += 2.0 * (S[H / 2].x * pmid.x + S[H / 2].y * pmid.y);
  }
  if (S) {
    const double lam = block_sum<NT>(acc, red) / (double)b;
    if (tid == 0) a.lam_per[(size_t)r * a.B + m] = lam;
  }
}

// Deflation by one component: lam = the median over the B per-sketch values
// lam_per[0..B-1] (every wave forms it, as k_median_scalar does; B <= 64),
// written to *lam_out by the first thread; S64[m][k] -= lam prod[m][k],
// S32 = (float)S64.  Whole waves only (blockDim a multiple of 64).
__global__ void k_spec_deflate(cx<double>* S64, cx<float>* S32, const cx<double>* prod, const double* lam_per,
                               int B, int H1, double* lam_out) {
  const int lane = threadIdx.x & 63;
  const double med = wave_median<double>(lane < B ? lam_per[lane] : 0.0, B);
  if (blockIdx.x == 0 && threadIdx.x == 0) *lam_out = med;
  const double cf = -1.0 * med;
  const size_t total = (size_t)B * H1;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    cx<double> s = S64[e];
    const cx<double> p = prod[e];
    s.x += cf * p.x;
    s.y += cf * p.y;
    S64[e] = s;
    if (S32) S32[e] = cx<float>{(float)s.x, (float)s.y};
  }
}

// S64[m][k] += sum_r coef_r prod[r][m][k]; S32 = (float)S64; coef_r = sign * lam[r].
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
__global__ __launch_bounds__(threads_for_h<double>(LOGB - 1)) void k_r2c64(const double* s_time,
                                                                     cx<double>* S64, cx<float>* S32,
                                                                     const cx<double>* twg,
                                                                     int accumulate) {
  constexpr int LOGH = LOGB - 1;
  constexpr int NT = threads_for_h<double>(LOGH);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  constexpr int PL = padded_len(H);
  __shared__ __align__(16) double re[2 * PL];
  double* im = re + PL;
  const Soa<double> buf{re, im};
  const int m = blockIdx.x;
  const Twid<double> tw{twg, twg + pass_table_len(H, NT)};
  const cx<double>* src = reinterpret_cast<const cx<double>*>(s_time + (size_t)m * b);
  for (int t = threadIdx.x; t < H; t += NT) buf.put(t, src[t]);
  __syncthreads();
  fft_soa<double, LOGH, NT, false>(buf, tw);
  cx<double>* S = S64 + (size_t)m * (H + 1);
  for (int k = threadIdx.x; k <= H; k += NT) {
    cx<double> X = r2c_post(buf.get(k & (H - 1)), buf.get((H - k) & (H - 1)), tw.w(k));
    if (accumulate) X = cadd(X, S[k]);
    S[k] = X;
    if (S32) S32[(size_t)m * (H + 1) + k] = cx<float>{(float)X.x, (float)X.y};
  }
}

template <int LOGB>
__global__ __launch_bounds__(threads_for_h<double>(LOGB - 1)) void k_c2r64(const cx<double>* S64,
                                                                     double* s_time,
                                                                     const cx<double>* twg) {
  constexpr int LOGH = LOGB - 1;
  constexpr int NT = threads_for_h<double>(LOGH);
  constexpr int b = 1 << LOGB;
  constexpr int H = b / 2;
  constexpr int PL = padded_len(H);
  __shared__ __align__(16) double re[2 * PL];
  double* im = re + PL;
  const Soa<double> buf{re, im};
  const int m = blockIdx.x;
  const Twid<double> tw{twg, twg + pass_table_len(H, NT)};
  const cx<double>* S = S64 + (size_t)m * (H + 1);
  for (int k = threadIdx.x; k < H; k += NT) buf.put(k, c2r_pack(S[k], S[H - k], tw.w(k)));
  __syncthreads();
  fft_soa<double, LOGH, NT, true>(buf, tw);
  double* dst = s_time + (size_t)m * b;
  const double scale = 2.0 / (double)b;
  for (int t = threadIdx.x; t < H; t += NT) {
    const cx<double> y = buf.get(t);
    dst[2 * t] = y.x * scale;
    dst[2 * t + 1] = y.y * scale;
  }
}

// ---------------------------------------------------------------------------
// Dense build, Eq. (1).  Work-group (slab, group): the G <= 2 sketches of
// `group` accumulate a contiguous slab of (i, j) fibres of T in LDS bins,
// then write the bins as one FP64 partial sum.  A wave takes four fibres
// T[i][j][:] at a time with its lanes along k in chunks of 64 (coalesced
// reads) and loads the next four while it scatters the current ones.  The
// offsets and signs of the fibres' first two modes come precomputed
// (k_fibre_offsets) and those of the third mode stay in registers, so every
// load of the loop is a buffer load from loop-invariant lane offsets.
//
// Bins are 64-bit fixed point: integer LDS atomics are an order of magnitude
// faster than floating-point ones on this chip, and integer sums do not
// depend on the order of the adds.  Each work-group scales its slab by 2^F,
// with F chosen from max |T| and the slab's element count so that no bin can
// overflow and no scaled entry reaches 2^50; a tensor with a non-finite
// entry writes NaN partials.
// ---------------------------------------------------------------------------
constexpr int kBuildMaxG = 2;

template <typename TIn>
struct BuildArgs {
  const TIn* T;
  int n, b, B, G;
  int nrange, lbr;            // bin ranges per sketch, log2 of their length
  const uint32_t* t3;         // third-mode table words of sketch m at t3 + m * t3s
  int t3s;
  const uint32_t* ef;         // [B][efs] codes of the fibres' first two modes
  long long efs;              // row length of ef (>= nfib + 4, multiple of 4)
  long long nfib;             // fibres: n^2, or the n(n+1)/2 pairs i <= j (SYM)
  long long pairs_per_slab;   // fibres per slab, a multiple of 4
  int nslab, ngroups;
  const unsigned long long* absmax;  // [nabs] per-block max |T| of k_absmax
  int nabs;
  double* partial;            // [ngroups][nslab][G][bins]
};

// A table entry (h << 1 | sign bit) as the byte offset of a 64-bit bin with
// the sign in bit 31: the sum of three such values is the bin's byte offset
// before the modulo (below 2^21) with the product of the signs in bit 31.
__device__ __forceinline__ uint32_t bin_code(uint32_t e) { return ((e >> 1) << 3) | (e << 31); }

// Colliding-hash table word (h << 2 | rotation q) as a code whose sums over
// three indices carry the summed positions from bit 4 and the summed
// rotations (at most 9) in bits 0-3: the complex bucket t = positions mod b
// is stored as real bins 2t (real part) and 2t + 1 (imaginary part), so a
// rotation r puts the value in bin 2t + (r & 1) with sign (-1)^(r >> 1).
__device__ __forceinline__ uint32_t sym_code(uint32_t e) { return ((e >> 2) << 4) | (e & 3u); }

// Pair p = j (j + 1) / 2 + i, i <= j.
__device__ inline void pair_of(long long p, int& i, int& j) {
  int jj = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
  while ((long long)(jj + 1) * (jj + 2) / 2 <= p) ++jj;
  while ((long long)jj * (jj + 1) / 2 > p) --jj;
  j = jj;
  i = (int)(p - (long long)jj * (jj + 1) / 2);
}

// ef[m][i n + j] = code of h1(i) + code of h2(j) for sketch m; the padding
// entries are zero.
__global__ void k_fibre_offsets(const uint32_t* __restrict__ hx, int n, int B, long long efs,
                                uint32_t* __restrict__ ef) {
  const long long nn = (long long)n * n;
  const long long total = (long long)B * efs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(e / efs);
    const long long p = e - (long long)m * efs;
    uint32_t v = 0;
    if (p < nn) {
      const int i = (int)(p / n), j = (int)(p - (long long)i * n);
      const uint32_t* hm = hx + (size_t)m * 3 * n;
      v = bin_code(hm[i]) + bin_code(hm[n + j]);
    }
    ef[e] = v;
  }
}

// out[blockIdx.x] = max |T| over this block's share of the `count` entries,
// as the bits of a non-negative double (Inf when the share holds a NaN or an
// Inf).  No atomics: the consumers reduce the per-block values themselves.
template <typename TIn>
__global__ __launch_bounds__(256) void k_absmax(const TIn* __restrict__ T, size_t count,
                                                unsigned long long* out) {
  double m = 0.0;
  bool bad = false;
  auto take = [&](double x) {
    x = fabs(x);
    bad |= !(x < __builtin_inf());
    m = fmax(m, x);
  };
  const size_t stride = (size_t)gridDim.x * 256;
  const size_t first = (size_t)blockIdx.x * 256 + threadIdx.x;
  size_t done = 0;
  if ((reinterpret_cast<uintptr_t>(T) & 15) == 0) {
    // 16-byte loads, four in flight per thread
    constexpr int W = 16 / (int)sizeof(TIn);
    using V = typename std::conditional<sizeof(TIn) == 4, float4, double2>::type;
    const V* Tv = reinterpret_cast<const V*>(T);
    const size_t nv = count / W;
    auto take_v = [&](const V& v) {
      if constexpr (sizeof(TIn) == 4) {
        take(v.x); take(v.y); take(v.z); take(v.w);
      } else {
        take(v.x); take(v.y);
      }
    };
    size_t e = first;
    for (; e + 3 * stride < nv; e += 4 * stride) {
      const V a0 = Tv[e], a1 = Tv[e + stride], a2 = Tv[e + 2 * stride], a3 = Tv[e + 3 * stride];
      take_v(a0); take_v(a1); take_v(a2); take_v(a3);
    }
    for (; e < nv; e += stride) take_v(Tv[e]);
    done = nv * W;
  }
  for (size_t e = done + first; e < count; e += stride) take((double)T[e]);
  if (bad) m = __builtin_inf();
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o));
  __shared__ double wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    out[blockIdx.x] = (unsigned long long)__double_as_longlong(fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3])));
}

// The largest of the np per-block values of k_absmax, in every thread of
// the work-group (red: 16 words of LDS; contains a barrier).
__device__ inline double reduce_absmax(const unsigned long long* p, int np, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v = fmax(v, __longlong_as_double((long long)p[i]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  v = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) v = fmax(v, red[w]);
  return v;
}

// Fixed-point scale exponent F of a slab of `count` entries with max |T| = m:
// count * m * 2^F < 2^62 (no bin overflows) and m * 2^F <= 2^50 (the
// rounding below is exact), clamped to where 2^F is a normal double.
__device__ inline int fixed_scale(double m, long long count) {
  int e2 = 0, em = 0;
  (void)frexp(m * (double)count * 2.0, &e2);
  (void)frexp(m, &em);
  return m > 0.0 ? max(-1000, min(1000, min(62 - e2, 50 - em))) : 0;
}

// round(x * 2^F) as a 64-bit two's-complement integer for |x * 2^F| <= 2^50:
// adding 1.5 * 2^52 rounds the product to an integer (ties to even, as
// rint) and leaves it in the low mantissa bits; the constant's low word is
// zero, so removing it touches only the high word.
__device__ __forceinline__ unsigned long long to_fixed(double x, double up) {
  const double d = fma(x, up, 6755399441055744.0);
  const uint32_t lo = (uint32_t)__double2loint(d);
  const uint32_t hi = (uint32_t)__double2hiint(d) - 0x43380000u;
  return ((unsigned long long)hi << 32) | lo;
}

// x with its sign flipped where bit 31 of s is set
__device__ __forceinline__ double signed_in(float x, uint32_t s) {
  return (double)__uint_as_float(__float_as_uint(x) ^ (s & 0x80000000u));
}
__device__ __forceinline__ double signed_in(double x, uint32_t s) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return __longlong_as_double((long long)(u ^ ((unsigned long long)(s & 0x80000000u) << 32)));
}

// ef[m][p] = sym_code(h(i)) + sym_code(h(j)) for pair p = (i, j) of sketch m
// (hq: [B][n] colliding-hash words); the padding entries are zero.
__global__ void k_pair_codes(const uint32_t* __restrict__ hq, int n, int B, long long efs,
                             uint32_t* __restrict__ ef) {
  const long long np = (long long)n * (n + 1) / 2;
  const long long total = (long long)B * efs;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(e / efs);
    const long long p = e - (long long)m * efs;
    uint32_t v = 0;
    if (p < np) {
      int i, j;
      pair_of(p, i, j);
      v = sym_code(hq[(size_t)m * n + i]) + sym_code(hq[(size_t)m * n + j]);
    }
    ef[e] = v;
  }
}

// One static pool of POOL 64-bit words holds the G sketches' bins.
// SPLIT: a sketch has more bins than one range (then G = 1).
// SYM: colliding-hash sketches of a symmetric tensor (Section 3.3, Eq. (5)):
// every index triple of one multiset falls in the same bucket with the same
// sign, so only the entries i <= j <= k are read, weighted by the number of
// distinct orderings of (i, j, k) (6, 3 or 1): the fibres T[i][j][:] of the
// pairs i <= j from k = j on (a fibre's chunks of 64 below j are skipped).
// Each sketch has 2b real bins (sym_code), and the sign of an entry is
// (-1)^(r >> 1) for its summed rotation r.
template <typename TIn, int POOL, bool SPLIT, bool SYM>
__global__ __launch_bounds__(1024) void k_build_dense(BuildArgs<TIn> a) {
  __shared__ __align__(16) unsigned long long pool[POOL];
  __shared__ double red[16];
  const int n = a.n, b = a.b, G = a.G;
  // Work-groups of one slab (all groups) are numbered consecutively within
  // one XCD (block ids are dealt round-robin over the 8 XCDs), so the slab's
  // re-reads for the other groups hit that XCD's L2.
  const int lin = blockIdx.x;
  const int xcd = lin & 7, r = lin >> 3;
  const int slab = (r / a.ngroups) * 8 + xcd;
  const int grp = r % a.ngroups;
  if (slab >= a.nslab) return;  // padding blocks of the XCD mapping
  // Work-group `grp` holds the bins of G consecutive (sketch, bin range)
  // pairs; with more than one range per sketch G is 1.
  const int g0 = grp * G;
  const int Gc = min(G, a.B * a.nrange - g0);
  const int br = 1 << a.lbr;
  const int sk0 = g0 / a.nrange, rq = g0 % a.nrange;
  unsigned long long* bins = pool;
  const int tid = threadIdx.x;
  for (int t = tid; t < G * br; t += blockDim.x) bins[t] = 0ull;

  // A slab is a range of fibres; with SYM its items of NF pairs are dealt
  // round-robin over the slabs instead (the pairs of small j have entries in
  // more blocks of k than those of large j, so ranges would be unbalanced).
  const long long p0 = SYM ? 0 : (long long)slab * a.pairs_per_slab;
  const long long p1 = SYM ? a.nfib : min(a.nfib, p0 + a.pairs_per_slab);
  const double m = reduce_absmax(a.absmax, a.nabs, red);  // contains a barrier
  const bool bad = !(m < __builtin_inf());
  const int F = bad ? 0 : fixed_scale(SYM ? 6.0 * m : m, (SYM ? a.pairs_per_slab : p1 - p0) * n);
  const double up = ldexp(1.0, F), down = ldexp(1.0, -F);
  __syncthreads();

  if (!bad) {
    const int lane = tid & 63;
    const int nw = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    constexpr int NF = 4;   // fibres per item
    constexpr int NC = 4;   // chunks of 64 lanes along k per item
    constexpr int GM = kBuildMaxG;
    constexpr unsigned SZ = sizeof(TIn);
    const uint32_t pmask = ((uint32_t)b - 1u) << (SYM ? 4 : 3);
    const uint32_t lmask = ((uint32_t)br - 1u) << 3;
    const long long step = SYM ? (long long)NF * a.nslab * nw : (long long)NF * nw;
    const __amdgpu_buffer_rsrc_t efr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t*>(a.ef + (size_t)sk0 * a.efs), 0, (int)(Gc * a.efs * 4), kBufferWord3);
    // The item of fibres q .. q+3: their ef words (per sketch), entries and
    // (SYM) which of them are diagonal pairs and their second index j.
    struct Item {
      uint32_t ef[GM][NF];
      TIn x[NF][NC];
      uint32_t diag;
      int jf[NF];
    };
    for (int kb = 0; kb < n; kb += 64 * NC) {
      // (SYM) pairs (i, j) with j >= kb + 64 NC have no entry k >= j in this
      // block of k: they come last in pair order and are not visited
      const long long pe =
          SYM ? min(p1, (long long)(kb + 64 * NC) * (long long)(kb + 64 * NC + 1) / 2) : p1;
      unsigned voff[NC];
      bool kin[NC];
      uint32_t e3[GM][NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int k = kb + 64 * c + lane;
        kin[c] = k < n;
        voff[c] = (unsigned)min(k, n - 1) * SZ;
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          if (g < Gc) {
            const uint32_t w = a.t3[(size_t)(sk0 + g) * a.t3s + min(k, n - 1)];
            e3[g][c] = SYM ? sym_code(w) : bin_code(w);
          } else {
            e3[g][c] = 0u;
          }
        }
      }
      // Every variable offset is a lane offset, which the buffer range check
      // covers: a fibre past the slab gets a resource of zero bytes.
      auto load = [&](long long q, Item& it) {
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          if (g < Gc) {
            const auto w = __builtin_amdgcn_raw_buffer_load_b128(
                efr, (unsigned)((g * a.efs + min(q, a.efs - NF)) * 4), 0u, 0);
            it.ef[g][0] = w[0];
            it.ef[g][1] = w[1];
            it.ef[g][2] = w[2];
            it.ef[g][3] = w[3];
          }
        }
        int pi = 0, pj = 0;
        if (SYM) pair_of(min(q, a.nfib - 1), pi, pj);
        it.diag = 0u;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
          const bool live = q + f < pe;
          long long row = q + f;
          if (SYM) {
            row = (long long)pi * n + pj;
            it.diag |= (pi == pj ? 1u : 0u) << f;
            it.jf[f] = pj;
            if (++pi > pj) {
              ++pj;
              pi = 0;
            }
          }
          const __amdgpu_buffer_rsrc_t tr = __builtin_amdgcn_make_buffer_rsrc(
              const_cast<TIn*>(a.T) + (size_t)(live ? row : 0) * n, 0, live ? (int)(n * SZ) : 0,
              kBufferWord3);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            // (SYM) a chunk wholly below k = j is never used: not loaded (wave-uniform)
            if (SYM && kb + 64 * c + 63 < it.jf[f]) {
              it.x[f][c] = TIn(0);
              continue;
            }
            if constexpr (sizeof(TIn) == 4)
              it.x[f][c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(tr, voff[c], 0u, 0));
            else
              it.x[f][c] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(tr, voff[c], 0u, 0));
          }
        }
      };
      long long q0 = SYM ? (long long)NF * (slab + (long long)a.nslab * wv) : p0 + NF * wv;
      Item cur;
      load(q0, cur);
      while (q0 < pe) {
        const long long qn = q0 + step;
        Item nxt;
        load(qn, nxt);
        const int nf = (int)min((long long)NF, pe - q0);
#pragma unroll
        for (int g = 0; g < GM; ++g) {
          if (g < Gc) {
            const uint32_t gbase = SPLIT ? 0u : (uint32_t)g * (uint32_t)br * 8u;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
              if (f < nf) {
                // orderings of (i, j, k): 6 for i < j < k, 3 with one equality, 1 for i = j = k
                const bool dg = SYM && ((cur.diag >> f) & 1u);
                const int jf = SYM ? cur.jf[f] : 0;
                const double wo = dg ? 3.0 * up : 6.0 * up, wj = dg ? up : 3.0 * up;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                  if (SYM && kb + 64 * c + 63 < jf) continue;  // wave-uniform: chunk below j
                  const int kk = kb + 64 * c + lane;
                  if (kin[c] && (!SYM || kk >= jf)) {
                    const double upf = !SYM ? up : (kk == jf ? wj : wo);
                    const uint32_t sg = cur.ef[g][f] + e3[g][c];
                    const uint32_t off = SYM ? ((sg & pmask) | ((sg & 1u) << 3)) : (sg & pmask);
                    const unsigned long long v =
                        to_fixed(signed_in(cur.x[f][c], SYM ? (sg << 30) : sg), upf);
                    if (SPLIT) {
                      if ((int)(off >> (a.lbr + 3)) == rq)
                        atomicAdd(reinterpret_cast<unsigned long long*>(
                                      reinterpret_cast<unsigned char*>(bins) + (off & lmask)),
                                  v);
                    } else {
                      atomicAdd(reinterpret_cast<unsigned long long*>(
                                    reinterpret_cast<unsigned char*>(bins) + (off | gbase)),
                                v);
                    }
                  }
                }
              }
            }
          }
        }
        cur = nxt;
        q0 = qn;
      }
    }
  }
  __syncthreads();
  double* out = a.partial + ((size_t)grp * a.nslab + slab) * (size_t)G * br;
  for (int t = tid; t < Gc * br; t += blockDim.x)
    out[t] = bad ? __builtin_nan("") : (double)(long long)bins[t] * down;
}

// s_time[m][t] = sum over slabs of the partial bins (FP64); bucket t of
// sketch m lives in range t >> lbr of virtual sketch m * nrange + range.
__global__ void k_build_reduce(const double* partial, double* s_time, int b, int B, int G, int nslab,
                               int nrange, int lbr) {
  const size_t total = (size_t)B * b;
  const int br = 1 << lbr;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / b);
    const int t = (int)(e - (size_t)m * b);
    const int vs = m * nrange + (t >> lbr);
    const int grp = vs / G, g = vs - grp * G;
    const double* p = partial + ((size_t)grp * nslab * G + g) * br + (t & (br - 1));
    double s = 0.0;
    int sl = 0;
    for (; sl + 8 <= nslab; sl += 8) {  // eight loads in flight, summed in slab order
      double t8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) t8[q] = p[(size_t)(sl + q) * G * br];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += t8[q];
    }
    for (; sl < nslab; ++sl) s += p[(size_t)sl * G * br];
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
  __shared__ double bv[4];
  __shared__ int bt[4];
  __shared__ int s_tau;
  double best = 0.0;
  int bi = -1;
  for (int t = threadIdx.x; t < L; t += 256) {
    const double x = lam_med[t];
    const bool fin = (x == x) && x > -__builtin_inf() && x < __builtin_inf();
    if (fin && (bi < 0 || x > best)) {
      best = x;
      bi = t;
    }
  }
  // wave reduction: larger value wins, then the lower index
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ob = __shfl_down(best, o);
    const int oi = __shfl_down(bi, o);
    if (oi >= 0 && (bi < 0 || ob > best || (ob == best && oi < bi))) {
      best = ob;
      bi = oi;
    }
  }
  if ((threadIdx.x & 63) == 0) {
    bv[threadIdx.x >> 6] = best;
    bt[threadIdx.x >> 6] = bi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double b0 = 0.0;
    int t0 = -1;
    for (int w = 0; w < 4; ++w) {
      if (bt[w] < 0) continue;
      if (t0 < 0 || bv[w] > b0 || (bv[w] == b0 && bt[w] < t0)) {
        b0 = bv[w];
        t0 = bt[w];
      }
    }
    s_tau = t0 < 0 ? 0 : t0;
    if (tau_out) *tau_out = s_tau;
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

template <typename R>
__global__ void k_widen(const R* src, double* dst, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    dst[e] = (double)src[e];
}

// ---------------------------------------------------------------------------
// Gradient of f(u) = med_m <s^(m), s^(m)(u (x) u (x) u)>, one work-group per
// restart: the median's members (rank (B-1)/2, and B/2 for even B, ties by
// sketch index) and grad = scale * mean over the members of the sum of the
// three mode read-offs V0 + V1 + V2 ([L][B][n] each).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_tuuu_grad(const double* lam_per, const R* V0, const R* V1,
                                                   const R* V2, const R* scale, int n, int B,
                                                   double* f_med, R* grad) {
  __shared__ int sel[2];
  __shared__ int any_nan;
  const int tau = blockIdx.x;
  const double* lp = lam_per + (size_t)tau * B;
  if (threadIdx.x == 0) {
    sel[0] = 0;
    sel[1] = 0;
    any_nan = 0;
  }
  __syncthreads();
  const int ra = (B - 1) / 2, rb = B / 2;
  for (int m = threadIdx.x; m < B; m += blockDim.x) {
    const double x = lp[m];
    int r = 0;
    for (int j = 0; j < B; ++j) r += (lp[j] < x) || (lp[j] == x && j < m);
    if (r == ra) sel[0] = m;
    if (r == rb) sel[1] = m;
    if (__builtin_isnan(x)) any_nan = 1;
  }
  __syncthreads();
  const int m0 = sel[0], m1 = sel[1];
  const bool two = (B & 1) == 0;
  if (threadIdx.x == 0)
    f_med[tau] = any_nan ? __builtin_nan("") : (two ? 0.5 * (lp[m0] + lp[m1]) : lp[m0]);
  const double sc = (scale ? (double)scale[tau] : 1.0) * (two ? 0.5 : 1.0);
  const size_t r0 = ((size_t)tau * B + m0) * n, r1 = ((size_t)tau * B + m1) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double g = (double)V0[r0 + i] + (double)V1[r0 + i] + (double)V2[r0 + i];
    if (two) g += (double)V0[r1 + i] + (double)V1[r1 + i] + (double)V2[r1 + i];
    grad[(size_t)tau * n + i] = (R)(sc * g);
  }
}

// ---------------------------------------------------------------------------
// Sketched CP loss from the residual spectra R = S - sum_i lam_i prod_j F(s_j u_i):
// loss = (1/B) sum_m ||r^(m)||^2 = (1/(B b)) sum_m sum_k w_k |R_k|^2 (Parseval
// on the half spectrum: w = 1 at k = 0 and k = b/2, 2 elsewhere).  One
// work-group; fixed reduction order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_parseval_loss(const cx<double>* R64, int B, int b,
                                                        double* loss) {
  __shared__ double red[16];
  const int H1 = b / 2 + 1;
  double acc = 0.0;
  for (size_t e = threadIdx.x; e < (size_t)B * H1; e += 1024) {
    const int k = (int)(e % H1);
    const cx<double> z = R64[e];
    const double w = (k == 0 || k == H1 - 1) ? 1.0 : 2.0;
    acc += w * (z.x * z.x + z.y * z.y);
  }
  const double s = block_sum<1024>(acc, red);
  if (threadIdx.x == 0) loss[0] = s / ((double)B * (double)b);
}

// Gradients of the sketched CP loss, one work-group per component i:
//   grad_lam[i] = -(2/B) scale sum_m lam_per[i][m]        (lam_per = <r^(m), s^(m)(u_i^(x)3)>)
//   grad_U[i]   = -(2/B) scale lam_i sum_m (V0 + V1 + V2)[i][m]
template <typename R>
__global__ __launch_bounds__(256) void k_cp_grad(const double* lam_per, const R* V0, const R* V1,
                                                 const R* V2, const R* lam, const R* scale, int n,
                                                 int B, R* grad_lam, R* grad_U) {
  const int i = blockIdx.x;
  const double sc = (scale ? (double)scale[0] : 1.0) * (-2.0 / (double)B);
  if (grad_lam && threadIdx.x == 0) {
    double g = 0.0;
    for (int m = 0; m < B; ++m) g += lam_per[(size_t)i * B + m];
    grad_lam[i] = (R)(sc * g);
  }
  if (grad_U) {
    const double f = sc * (double)lam[i];
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      double g = 0.0;
      for (int m = 0; m < B; ++m) {
        const size_t o = ((size_t)i * B + m) * n + c;
        g += (double)V0[o] + (double)V1[o] + (double)V2[o];
      }
      grad_U[(size_t)i * n + c] = (R)(f * g);
    }
  }
}

// ===========================================================================
// Sketch of the whitened LDA moment M3(W,W,W) from document word counts
// (Appendix D).  Per document d with counts n (length m >= 3) and p = W^T n:
//   c_d  = 1 / (m (m-1)(m-2)),  c'_d = 1 / (m (m-1))
//   doc term   c_d p^(x)3 - a c'_d (p p q + p q p + q p p)           (a = alpha0/(alpha0+2))
// and, through the per-word sums g_i = sum_d c_d n_di, g'_i = sum_d c'_d n_di,
// R_i = sum_d c_d n_di p_d (w_i the i-th row of W),
//   word term  2 g_i w_i^(x)3 - (w w R_i + w R_i w + R_i w w) + a g'_i (w w q + w q w + q w w),
// then M3 = (sum of all terms) / D + c q^(x)3 with q = W^T M1.  Every rank-1
// term x (x) y (x) z is sketched as F(s1 x) F(s2 y) F(s3 z) (Eq. (2)).
// ===========================================================================

// Matrix-core steps of 16 x 16 x 4 (k = 4): lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; output v < 4 of lane l is D[row(l / 16, v)][l % 16], with
// row = 4 (l / 16) + v in FP32 and (l / 16) + 4 v in FP64 (measured on gfx950).
typedef float mfma_f32x4 __attribute__((ext_vector_type(4)));
typedef double mfma_f64x4 __attribute__((ext_vector_type(4)));
template <typename R>
struct Mfma16;
template <>
struct Mfma16<float> {
  using acc = mfma_f32x4;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return 4 * kq + v; }
};
template <>
struct Mfma16<double> {
  using acc = mfma_f64x4;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int v) { return kq + 4 * v; }
};

// p_d = W^T n_d for 16 documents per work-group as one dense product on the
// matrix cores, and the document coefficients.  The tile's nonzeros e (their
// documents' CSR ranges, concatenated) are the inner dimension: A[r][e] is the
// count of e when e belongs to the tile's document r (zero otherwise) and
// B[e][c] = W[word(e)][c], so P_tile = A B.  Each MFMA step takes four
// nonzeros; wave w owns the column blocks w and w + 4 of 16 columns (K <= 128).
// Each lane follows one nonzero per step and keeps its document row by
// walking the tile's CSR bounds forward.  Counts are integers, exact in R; the
// document length m_d comes from the same A values.
template <typename R>
__global__ __launch_bounds__(256) void k_doc_project(const int32_t* rowptr, const int32_t* col,
                                                     const int32_t* cnt, int D, int K, const R* W,
                                                     R* P, double* cd, double* cpd, double* invm) {
  using M = Mfma16<R>;
  __shared__ int bnd[17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int c0 = wave * 16 + r16, c1 = c0 + 64;
  const bool v0 = c0 < K, v1 = c1 < K;
  const int ntile = (D + 15) >> 4;
  for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
    const int d0 = t << 4;
    __syncthreads();  // the previous tile's readers of bnd are done
    if (threadIdx.x <= 16) bnd[threadIdx.x] = rowptr[min(d0 + (int)threadIdx.x, D)];
    __syncthreads();
    const int lo = bnd[0], hi = bnd[16];
    typename M::acc acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    R msum = 0;
    int e = lo + kq;
    int row = 0;
    while (row < 16 && e >= bnd[row + 1]) ++row;
    int e0 = lo;
    // four steps (16 nonzeros) per round while all are in range
    for (; e0 + 16 <= hi; e0 += 16) {
      int w[4], n[4], rw[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        w[u] = col[e + 4 * u];
        n[u] = cnt[e + 4 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        rw[u] = row;
        e += 4;
        while (row < 16 && e >= bnd[row + 1]) ++row;
      }
      R b0[4], b1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        b0[u] = v0 ? W[(size_t)w[u] * K + c0] : (R)0;
        b1[u] = v1 ? W[(size_t)w[u] * K + c1] : (R)0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const R a = rw[u] == r16 ? (R)n[u] : (R)0;
        acc0 = M::mac(a, b0[u], acc0);
        acc1 = M::mac(a, b1[u], acc1);
        msum += a;
      }
    }
    for (; e0 < hi; e0 += 4) {
      const bool ok = e < hi;
      const int es = ok ? e : lo;
      const int w = col[es], n = cnt[es];
      const R a = (ok && row == r16) ? (R)n : (R)0;
      const R b0 = v0 ? W[(size_t)w * K + c0] : (R)0;
      const R b1 = v1 ? W[(size_t)w * K + c1] : (R)0;
      acc0 = M::mac(a, b0, acc0);
      acc1 = M::mac(a, b1, acc1);
      msum += a;
      e += 4;
      while (row < 16 && e >= bnd[row + 1]) ++row;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int d = d0 + M::row(kq, v);
      if (d < D) {
        if (v0) P[(size_t)d * K + c0] = acc0[v];
        if (v1) P[(size_t)d * K + c1] = acc1[v];
      }
    }
    if (wave == 0) {
      // lanes r16, r16 + 16, r16 + 32, r16 + 48 hold parts of document r16's length
      double m = (double)msum;
      m += __shfl_xor(m, 16);
      m += __shfl_xor(m, 32);
      const int d = d0 + r16;
      if (kq == 0 && d < D) {
        const bool keep = m >= 3.0;  // documents with fewer than three words are dropped
        cd[d] = keep ? 1.0 / (m * (m - 1.0) * (m - 2.0)) : 0.0;
        cpd[d] = keep ? 1.0 / (m * (m - 1.0)) : 0.0;
        invm[d] = keep ? 1.0 / m : 0.0;
      }
    }
  }
}

// Partial sums of p_d / m_d and of the kept-document count over a range of
// documents: part[g][k] for k < K, part[g][K] = count.
template <typename R>
__global__ __launch_bounds__(256) void k_doc_q_partial(const R* P, const double* invm, int D, int K,
                                                       int per, double* part) {
  const int g = blockIdx.x;
  const int d0 = g * per, d1 = min(D, d0 + per);
  for (int k = threadIdx.x; k <= K; k += blockDim.x) {
    double acc = 0.0;
    for (int d = d0; d < d1; ++d) {
      const double w = invm[d];
      if (k < K) acc += (double)P[(size_t)d * K + k] * w;
      else acc += w > 0.0 ? 1.0 : 0.0;
    }
    part[(size_t)g * (K + 1) + k] = acc;
  }
}

// q = (sum of partials) / D_eff, and D_eff itself: one work-group of 256
// threads per column k <= K (column K is the kept-document count, which every
// work-group sums again for its division); fixed strided sums and a fixed tree.
__global__ __launch_bounds__(256) void k_doc_q_final(const double* part, int G, int K, double* q,
                                                     double* deff) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  double s = 0.0, c = 0.0;
  for (int g = threadIdx.x; g < G; g += 256) {
    s += part[(size_t)g * (K + 1) + k];
    c += part[(size_t)g * (K + 1) + K];
  }
  s = block_sum<256>(s, red);
  const double D = block_sum<256>(c, red);
  if (threadIdx.x == 0) {
    if (k < K) q[k] = D > 0.0 ? s / D : 0.0;
    else deff[0] = D;
  }
}

// packed[e] = (d << 32) | cnt[e] for the nonzeros e of document d, the values
// the sort by word carries along; one wave per document, so that a
// document's writes are consecutive.
__global__ void k_pack_entries(const int32_t* rowptr, const int32_t* cnt, int D, unsigned long long* packed) {
  const int lane = threadIdx.x & 63, wpb = blockDim.x >> 6;
  for (int d = blockIdx.x * wpb + (threadIdx.x >> 6); d < D; d += gridDim.x * wpb) {
    const int lo = rowptr[d], hi = rowptr[d + 1];
    for (int e = lo + lane; e < hi; e += 64)
      packed[e] = ((unsigned long long)(uint32_t)d << 32) | (uint32_t)cnt[e];
  }
}

// colptr[i] = first position of word i in the sorted word ids (binary search).
__global__ void k_col_bounds(const int32_t* skeys, int nnz, int V, int32_t* colptr) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= V; i += gridDim.x * blockDim.x) {
    int lo = 0, hi = nnz;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (skeys[mid] < i) lo = mid + 1;
      else hi = mid;
    }
    colptr[i] = lo;
  }
}

// sdoc[e], scnt[e]: document and count of the e-th nonzero in word order
// (packed: the values of k_pack_entries sorted by word, stable in document
// order), so that the per-word kernels read them without a chain of
// dependent loads.
__global__ void k_unpack_entries(const unsigned long long* packed, int nnz, int32_t* sdoc, int32_t* scnt) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += gridDim.x * blockDim.x) {
    const unsigned long long v = packed[e];
    sdoc[e] = (int32_t)(v >> 32);
    scnt[e] = (int32_t)(uint32_t)v;
  }
}

// Per-word sums over the documents containing the word (in document order):
// R_i = sum_d c_d n_di p_d, g_i = sum_d c_d n_di, g'_i = sum_d c'_d n_di.
// wcd[d] = (c_d, c'_d), packed so that a document costs one load of them.
template <typename R>
__global__ __launch_bounds__(64) void k_word_accum(const int32_t* sdoc, const int32_t* scnt,
                                                   const int32_t* colptr, const R* P, const double2* wcd,
                                                   int V, int K, R* Rw, double* g, double* gp) {
  // sdoc, scnt: document and count of each nonzero in word order.  One wave
  // per word, two columns per lane (k and k + 64), sixteen documents per step:
  // 32 loads of P in flight per lane (sixteen partial sums per column), and the
  // next step's document indices loaded with this step's rows.
  constexpr int U = 16, CPT = 2;
  for (int w = blockIdx.x; w < V; w += gridDim.x) {
    const int lo = colptr[w], hi = colptr[w + 1];
    for (int kb = 0; kb < K; kb += CPT * (int)blockDim.x) {
      int kc[CPT];
      bool kv[CPT];
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        const int k = kb + (int)threadIdx.x + j * (int)blockDim.x;
        kv[j] = k < K;
        kc[j] = kv[j] ? k : K - 1;
      }
      double acc[CPT][U], ga = 0.0, gc = 0.0;
#pragma unroll
      for (int j = 0; j < CPT; ++j)
#pragma unroll
        for (int u = 0; u < U; ++u) acc[j][u] = 0.0;
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
        double n[U], c[U], c2[U];
        R p[CPT][U];
        int d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          d[u] = dn[u];
          n[u] = (double)nn[u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
          for (int j = 0; j < CPT; ++j) p[j][u] = P[(size_t)d[u] * K + kc[j]];
          const double2 wd = wcd[d[u]];
          c[u] = wd.x;
          c2[u] = wd.y;
        }
        if (e + 2 * U <= hi) load_idx(e + U);
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
          for (int j = 0; j < CPT; ++j) acc[j][u] += c[u] * n[u] * (double)p[j][u];
          ga += c[u] * n[u];
          gc += c2[u] * n[u];
        }
      }
      for (; e < hi; ++e) {
        const int d = sdoc[e];
        const double n = (double)scnt[e];
        const double2 wd = wcd[d];
        const double c = wd.x;
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[j][0] += c * n * (double)P[(size_t)d * K + kc[j]];
        ga += c * n;
        gc += wd.y * n;
      }
#pragma unroll
      for (int j = 0; j < CPT; ++j) {
        // the partial sums pairwise, in a fixed order
#pragma unroll
        for (int h = 1; h < U; h *= 2)
#pragma unroll
          for (int u = 0; u < U; u += 2 * h) acc[j][u] += acc[j][u + h];
        if (kv[j]) Rw[(size_t)w * K + kc[j]] = (R)acc[j][0];
      }
      if (kb == 0 && threadIdx.x == 0) {
        g[w] = ga;
        gp[w] = gc;
      }
    }
  }
}

// Half spectra F(s_j q) of one vector for every sketch m and mode j:
// Qs[m][j][k], k = 0..H; one work-group per (m, j).
template <typename R, int LOGB>
__global__ __launch_bounds__(threads_for_h<R>(LOGB - 1)) void k_mode_spectra(
    const uint32_t* hxs, const uint32_t* ord, int n, const double* q, const cx<R>* twg, cx<R>* Qs) {
  constexpr int LOGH = LOGB - 1;
  constexpr int NT = threads_for_h<R>(LOGH);
  constexpr int H = 1 << LOGH;
  constexpr int PL = padded_len(H);
  __shared__ __align__(16) R re[2 * PL];
  R* im = re + PL;
  const Soa<R> buf{re, im};
  const int m = blockIdx.x, j = blockIdx.y;
  const size_t tb = ((size_t)m * 3 + j) * n;
  const Twid<R> tw{twg, twg + pass_table_len(H, NT)};
  for (int t = threadIdx.x; t < 2 * PL; t += NT) re[t] = R(0);
  __syncthreads();
  auto getu = [&](uint32_t i) -> R { return (R)q[i]; };
  auto store = [&](uint32_t t, R v) { store_packed(buf, t, v); };
  count_sketch<R>(hxs + tb, ord + tb, n, NT, getu, store);
  __syncthreads();
  fft_soa<R, LOGH, NT, false, false>(buf, tw);
  cx<R>* out = Qs + ((size_t)m * 3 + j) * (H + 1);
  for (int k = threadIdx.x; k <= H; k += NT)
    out[k] = r2c_post(buf.get(k & (H - 1)), buf.get((H - k) & (H - 1)), tw.w(k));
}

struct TermArgs {
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B;                // n = K, the whitened dimension
  int nitem, per;          // items, items per work-group
  const void* X;           // R[nitem][n]: p_d (documents) or w_i (words)
  const void* Y;           // R[nitem][n]: R_i (words) or null
  const double* arrA;      // [nitem]
  const double* arrB;      // [nitem]
  double sa, sb, gam;      // alpha = sa arrA, beta = sb arrB, gamma (Y terms)
  const void* Qs;          // cx<R>[B][3][H+1]
  const void* twg;
  cx<double>* part;        // [B][nchunk][H+1]
};

// Sum over a range of items of
//   alpha F1x F2x F3x + beta (F1x F2x Q3 + F1x Q2 F3x + Q1 F2x F3x)
//   + gamma (F1y F2x F3x + F1x F2y F3x + F1x F2x F3y)
// for sketch m, in FP64 registers; one work-group per (m, chunk).  The three
// products are built mode by mode with the product rule, P = prod_j F_j x,
// S = sum_j Q_j prod_{i != j} F_i x, Dy = sum_j F_j y prod_{i != j} F_i x, so
// only P, S (and Dy) are held.  The owned bins are processed in NPART rounds
// (the transforms are redone per round) to bound the registers.
template <typename R, int LOGB, bool HAS_Y, int NPART>
__global__ __launch_bounds__(threads_for_h<R>(LOGB - 1)) void k_terms(TermArgs a) {
  constexpr int LOGH = LOGB - 1;
  constexpr int NT = threads_for_h<R>(LOGH);
  constexpr int H = 1 << LOGH;
  constexpr int PL = padded_len(H);
  constexpr int PK = (H / 2 + NT - 1) / NT;
  constexpr int PKP = (PK + NPART - 1) / NPART;
  // every slot of every round is a valid bin pair when the pairs split evenly
  constexpr bool ALL = (H / 2) % NT == 0 && PK % NPART == 0;
  // With a last pass of radix 2 the transforms stop before it and the bins
  // are formed from its inputs: Z[k] = A[k] + W_H^k A[k + H/2] and, for
  // j = H/2 - k, Z[H-k] = A[j] + conj(W_H^k) A[j + H/2], W_H^k = (W_b^k)^2.
  constexpr bool FUSE = fft_last_radix(H, NT) == 2 && H >= 64;
  extern __shared__ __align__(16) unsigned char lds[];
  R* re = reinterpret_cast<R*>(lds);
  R* im = re + PL;
  const int n = a.n;
  R* xv = reinterpret_cast<R*>(lds + align16(sizeof(R) * 2 * (size_t)PL));
  R* yv = xv + ((n + 3) & ~3);
  uint32_t* stab = reinterpret_cast<uint32_t*>(yv + ((n + 3) & ~3));  // [3][2][n]
  const Soa<R> buf{re, im};
  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const int chunk = blockIdx.y;
  const size_t tb = (size_t)m * 3 * n;
  const Twid<R> tw{reinterpret_cast<const cx<R>*>(a.twg),
                   reinterpret_cast<const cx<R>*>(a.twg) + pass_table_len(H, NT)};
  const cx<R>* Q = reinterpret_cast<const cx<R>*>(a.Qs) + (size_t)m * 3 * (H + 1);
  const R* X = reinterpret_cast<const R*>(a.X);
  const R* Y = reinterpret_cast<const R*>(a.Y);
  for (int e = tid; e < n; e += NT)
    for (int j = 0; j < 3; ++j) {
      stab[(2 * j) * n + e] = a.hxs[tb + (size_t)j * n + e];
      stab[(2 * j + 1) * n + e] = a.ord[tb + (size_t)j * n + e];
    }
  const int i0 = chunk * a.per, i1 = min(a.nitem, i0 + a.per);
  cx<double>* out = a.part + ((size_t)m * gridDim.y + chunk) * (H + 1);
  auto fft_mode = [&](const R* vec, int j) {
    zero_lds<NT>(re, 2 * PL * (int)sizeof(R));
    __syncthreads();
    auto getu = [&](uint32_t i) -> R { return vec[i]; };
    auto store = [&](uint32_t t, R v) { store_packed(buf, t, v); };
    count_sketch<R>(stab + (2 * j) * n, stab + (2 * j + 1) * n, n, NT, getu, store);
    __syncthreads();
    fft_soa<R, LOGH, NT, false, false, FUSE>(buf, tw);
  };
  // Z[k] and Z[H-k] for 0 <= k < H/2 (Z[H] = Z[0]), and Z[H/2]; w = W_b^k
  auto zpair = [&](int k, cx<R> w, cx<R>& Za, cx<R>& Zb) {
    if constexpr (FUSE) {
      const cx<R> wH = cmul(w, w);
      Za = cadd(buf.get(k), cmul(wH, buf.get(k + H / 2)));
      Zb = k == 0 ? Za : cadd(buf.get(H / 2 - k), cmulc(buf.get(H - k), wH));
    } else {
      Za = buf.get(k);
      Zb = buf.get((H - k) & (H - 1));
    }
  };
  auto zmid = [&]() -> cx<R> { return FUSE ? csub(buf.get(0), buf.get(H / 2)) : buf.get(H / 2); };
  // owned bin pair (k, H-k) of slot s in round `part`; k < H/2 when valid
  auto bin_k = [&](int part, int s) -> int {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t + (part * PKP + s) * NT;
  };
  auto addc = [](cx<double>& acc, double c, cx<R> v) {
    acc.x += c * (double)v.x;
    acc.y += c * (double)v.y;
  };
  // Spectra of the transform in the buffer at the owned bins: X[k] and X[H-k]
  // (W_b^{H-k} = -conj W_b^k, since W_b^H = -1), and X[H/2] on thread 0.
  auto spectra = [&](int part, const cx<R>* w, cx<R>* X0, cx<R>* X1, cx<R>& Xm) {
#pragma unroll
    for (int s = 0; s < PKP; ++s) {
      const int k = bin_k(part, s);
      if (!ALL && k >= H / 2) break;
      cx<R> Za, Zb;
      zpair(k, w[s], Za, Zb);
      X0[s] = r2c_post(Za, Zb, w[s]);
      X1[s] = r2c_post(Zb, Za, cx<R>{-w[s].x, w[s].y});
    }
    if (tid == 0 && part == 0) {
      const cx<R> Z = zmid();
      Xm = r2c_post(Z, Z, cx<R>{R(0), R(-1)});
    }
  };
  // prefetch of the next item's vector and weights (threads e < n, e < NT)
  auto load_item = [&](int it, R& x, R& y, double& al, double& be) {
    if (it < i1) {
      if (tid < n) {
        x = X[(size_t)it * n + tid];
        if (HAS_Y) y = Y[(size_t)it * n + tid];
      }
      al = a.sa * a.arrA[it];
      be = a.sb * a.arrB[it];
    }
  };
#pragma unroll 1
  for (int part = 0; part < NPART; ++part) {
    cx<double> acc0[PKP], acc1[PKP], accm = {0.0, 0.0};
#pragma unroll
    for (int s = 0; s < PKP; ++s) acc0[s] = acc1[s] = cx<double>{0.0, 0.0};
    cx<R> wv[PKP];  // W_b^k of the owned bins, the same for every item and mode
#pragma unroll
    for (int s = 0; s < PKP; ++s) {
      const int k = bin_k(part, s);
      if (!ALL && k >= H / 2) break;
      wv[s] = tw.w(k);
    }
    R xn = R(0), yn = R(0);
    double alpha_n = 0.0, beta_n = 0.0;
    load_item(i0, xn, yn, alpha_n, beta_n);
#pragma unroll 1
    for (int it = i0; it < i1; ++it) {
      const double alpha = alpha_n, beta = beta_n;
      __syncthreads();  // the previous item's readers of xv / yv are done
      if (tid < n) {
        xv[tid] = xn;
        if (HAS_Y) yv[tid] = yn;
      }
      for (int e = tid + NT; e < n; e += NT) {
        xv[e] = X[(size_t)it * n + e];
        if (HAS_Y) yv[e] = Y[(size_t)it * n + e];
      }
      load_item(it + 1, xn, yn, alpha_n, beta_n);
      if (alpha == 0.0 && beta == 0.0) continue;  // uniform: an empty word or a dropped document
      cx<R> P0[PKP], P1[PKP], S0[PKP], S1[PKP], D0[PKP], D1[PKP], Pm, Sm, Dm;
      // One mode: F_j x (and F_j y) at the owned bins, then the product rule.
      auto mode = [&](int j, auto first) {
        constexpr bool FIRST = decltype(first)::value;
        const cx<R>* Qj = Q + (size_t)j * (H + 1);
        fft_mode(xv, j);
        cx<R> qa[PKP], qb[PKP], qm = {R(0), R(0)};
        auto load_q = [&]() {
#pragma unroll
          for (int s = 0; s < PKP; ++s) {
            const int k = bin_k(part, s);
            if (!ALL && k >= H / 2) break;
            qa[s] = Qj[k];
            qb[s] = Qj[H - k];
          }
          if (tid == 0 && part == 0) qm = Qj[H / 2];
        };
        if (!HAS_Y) load_q();  // in flight while the spectra are formed
        cx<R> F0[PKP], F1[PKP], Fm = {R(0), R(0)};
        spectra(part, wv, F0, F1, Fm);
        __syncthreads();
        cx<R> G0[PKP], G1[PKP], Gm = {R(0), R(0)};  // F_j y
        if constexpr (HAS_Y) {
          fft_mode(yv, j);
          load_q();
          spectra(part, wv, G0, G1, Gm);
          __syncthreads();
        }
        auto step = [&](cx<R>& P, cx<R>& S, cx<R>& Dy, cx<R> F, cx<R> G, cx<R> q) {
          if constexpr (FIRST) {
            if (HAS_Y) Dy = G;
            S = q;
            P = F;
          } else {
            if (HAS_Y) Dy = cadd(cmul(Dy, F), cmul(P, G));
            S = cadd(cmul(S, F), cmul(P, q));
            P = cmul(P, F);
          }
        };
#pragma unroll
        for (int s = 0; s < PKP; ++s) {
          const int k = bin_k(part, s);
          if (!ALL && k >= H / 2) break;
          step(P0[s], S0[s], D0[s], F0[s], HAS_Y ? G0[s] : F0[s], qa[s]);
          step(P1[s], S1[s], D1[s], F1[s], HAS_Y ? G1[s] : F1[s], qb[s]);
        }
        if (tid == 0 && part == 0) step(Pm, Sm, Dm, Fm, HAS_Y ? Gm : Fm, qm);
      };
      mode(0, std::true_type{});
#pragma unroll 1
      for (int j = 1; j < 3; ++j) mode(j, std::false_type{});
      const double gam = a.gam;
#pragma unroll
      for (int s = 0; s < PKP; ++s) {
        const int k = bin_k(part, s);
        if (!ALL && k >= H / 2) break;
        addc(acc0[s], alpha, P0[s]);
        addc(acc0[s], beta, S0[s]);
        addc(acc1[s], alpha, P1[s]);
        addc(acc1[s], beta, S1[s]);
        if (HAS_Y) {
          addc(acc0[s], gam, D0[s]);
          addc(acc1[s], gam, D1[s]);
        }
      }
      if (tid == 0 && part == 0) {
        addc(accm, alpha, Pm);
        addc(accm, beta, Sm);
        if (HAS_Y) addc(accm, gam, Dm);
      }
    }
#pragma unroll
    for (int s = 0; s < PKP; ++s) {
      const int k = bin_k(part, s);
      if (!ALL && k >= H / 2) break;
      out[k] = acc0[s];
      out[H - k] = acc1[s];  // k = 0 pairs with the Nyquist bin H
    }
    if (tid == 0 && part == 0) out[H / 2] = accm;
  }
}

// S64[m][k] (+)= (sum of the document and word partials in chunk order) / D_eff
//              + c prod_j Qs[m][j][k];  S32 = (float) S64.
template <typename R>
__global__ void k_terms_final(const cx<double>* partD, int ncD, const cx<double>* partW, int ncW,
                              const cx<R>* Qs, const double* deff, double c3, int B, int H1,
                              int accumulate, cx<double>* S64, cx<float>* S32) {
  const size_t total = (size_t)B * H1;
  const double D = deff[0];
  const double invD = D > 0.0 ? 1.0 / D : 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / H1), k = (int)(e % H1);
    cx<double> s = {0.0, 0.0};
    for (int c = 0; c < ncD; ++c) {
      const cx<double> v = partD[((size_t)m * ncD + c) * H1 + k];
      s.x += v.x;
      s.y += v.y;
    }
    for (int c = 0; c < ncW; ++c) {
      const cx<double> v = partW[((size_t)m * ncW + c) * H1 + k];
      s.x += v.x;
      s.y += v.y;
    }
    const cx<R>* Qm = Qs + (size_t)m * 3 * H1;
    const cx<double> q1 = {(double)Qm[k].x, (double)Qm[k].y};
    const cx<double> q2 = {(double)Qm[H1 + k].x, (double)Qm[H1 + k].y};
    const cx<double> q3 = {(double)Qm[2 * H1 + k].x, (double)Qm[2 * H1 + k].y};
    const cx<double> qq = cmul(cmul(q1, q2), q3);
    cx<double> r = {s.x * invD + c3 * qq.x, s.y * invD + c3 * qq.y};
    if (accumulate) {
      r.x += S64[e].x;
      r.y += S64[e].y;
    }
    S64[e] = r;
    if (S32) S32[e] = cx<float>{(float)r.x, (float)r.y};
  }
}

__global__ void k_fill_u32(unsigned* p, unsigned v, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

}  // namespace tsk
