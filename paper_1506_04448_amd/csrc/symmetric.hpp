// Colliding-hash symmetric tensor sketches (Section 3.3, Eq. (5)) and the
// tensor power method on them (Appendix B).
//
// One hash h: [n] -> [b] and one complex sign sigma(i) = i^q(i), q in
// {0, 1, 2, 3}, per sketch.  The sketch of a symmetric tensor,
//   s(t) = sum over (h(i) + h(j) + h(k)) mod b == t of sigma(i) sigma(j) sigma(k) T_ijk,
// is complex; it is built from the entries with i <= j <= k, each weighted by
// the number of distinct permutations of its index triple (6, 3 or 1).  It is
// kept in the time domain (the T(I,u,u) read-off takes s at 3h(i)) and as a
// full complex spectrum of b points.
//
// T(I,u,u)_i is estimated by the read-off of Appendix B with weight 1/3 on all
// four terms:
//   v_i = (1/3) [ conj(sigma_i) (c_1 + c_2)[h_i] / 2 + conj(sigma_i^2) u_i c_3[2h_i]
//                 + conj(sigma_i^3) u_i^2 s[3h_i] ],
//   c_1 + c_2 = F^-1(S o (conj(U_1)^2 + conj(U_2))),  c_3 = F^-1(S o conj(U_1)),
//   U_1 = F(s_u), s_u(t) = sum_{h(i)=t} sigma_i u_i,
//   U_2 = F(s_2), s_2(t) = sum_{2h(i)=t} sigma_i^2 u_i^2   (positions mod b),
// and the power step keeps Re v_i.  T(u,u,u) is u . Re v (the estimate
// <s, s_X> of Appendix B equals it: sum_i u_i s_{Z_i} = 3 s_X).
#pragma once

#include "kernels.hpp"

namespace tsk {

// Table words: (position << 2) | rotation, rotation = the power of i.
__device__ __forceinline__ uint32_t sym_pos(uint32_t e) { return e >> 2; }
__device__ __forceinline__ int sym_rot(uint32_t e) { return (int)(e & 3u); }

// x * i^r
template <typename R>
__device__ __forceinline__ cx<R> rot(cx<R> x, int r) {
  switch (r & 3) {
    case 0: return x;
    case 1: return {-x.y, x.x};
    case 2: return {-x.x, -x.y};
    default: return {x.y, -x.x};
  }
}

// Deterministic complex count sketch from a table sorted by position (stable
// by index): the entries sharing a bucket are summed by one thread in
// increasing index order; store(bucket, sum).  Entry words carry the rotation
// of sigma^p; getx(i) is the real value x_i (u_i, u_i^2, ...).
template <typename R, typename GetX, typename Store>
__device__ __forceinline__ void sym_count_sketch(const uint32_t* __restrict__ srt, const uint32_t* __restrict__ ord,
                                                 int n, int nt, GetX getx, Store store) {
  for (int p = threadIdx.x; p < n; p += nt) {
    uint32_t e = srt[p];
    const uint32_t bk = sym_pos(e);
    if (p > 0 && sym_pos(srt[p - 1]) == bk) continue;
    cx<R> acc = {R(0), R(0)};
    int q = p;
    while (true) {
      acc = cadd(acc, rot(cx<R>{getx(ord[q]), R(0)}, sym_rot(e)));
      if (++q >= n) break;
      e = srt[q];
      if (sym_pos(e) != bk) break;
    }
    store(bk, acc);
  }
}

// ---- build ------------------------------------------------------------------

// The dense symmetric build is k_build_dense<..., SYM = true> (kernels.hpp).

// dst = src (+ dst when acc), doubles.
__global__ void k_add64(double* dst, const double* src, size_t count, int acc) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = acc ? dst[e] + src[e] : src[e];
}

// ---- FP64 complex transforms ------------------------------------------------

// Complex FFT of rows of N = 2^LOGN points, one work-group per row:
// out[row] = F(in[row]) (INV: the unnormalised inverse).  With DEC = 2 the
// row is the decimated subsequence in[row / 2][2 s + row % 2] of a 2N-point
// input (the two halves of a radix-2 split).
template <int LOGN, bool INV, int DEC>
__global__ __launch_bounds__(threads_for_h<double>(LOGN)) void k_c2c64(const cx<double>* in, cx<double>* out,
                                                                         const cx<double>* tw) {
  constexpr int N = 1 << LOGN;
  constexpr int NT = threads_for_h<double>(LOGN);
  constexpr int PL = padded_len(N);
  extern __shared__ __align__(16) unsigned char lds[];
  double* re = reinterpret_cast<double*>(lds);
  const Soa<double> buf{re, re + PL};
  const int row = blockIdx.x;
  const cx<double>* src = in + (size_t)(row / DEC) * N * DEC;
  const int par = row % DEC;
  for (int s = threadIdx.x; s < N; s += NT) buf.put(s, src[(size_t)s * DEC + par]);
  __syncthreads();
  const Twid<double> twd{tw, nullptr};
  fft_soa<double, LOGN, NT, INV>(buf, twd);
  cx<double>* dst = out + (size_t)row * N;
  for (int k = threadIdx.x; k < N; k += NT) dst[k] = buf.get(k);
}

// Radix-R combination of the R sub-transforms E_s = rows R r + s (N points
// each, s < R) of the residue classes s mod R into the RN-point transform of
// row r: X[k] = sum_s W^{s k} E_s[k mod N], W = e^{-2 pi i / RN} (conjugate for
// INV), W^x from the full-circle table of RN points.  Optional FP32 copy.
__global__ void k_c2c_combine(const cx<double>* half, cx<double>* out, cx<float>* out32, const cx<double>* wb,
                              int N, int R, int rows, int inv) {
  const int RN = R * N;
  const size_t total = (size_t)rows * RN;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / RN;
    const int k = (int)(e % RN);
    const int km = k & (N - 1);
    cx<double> x = half[(R * r) * N + km];
    for (int q = 1; q < R; ++q) {
      cx<double> w = wb[(int)(((long)q * k) & (RN - 1))];
      if (inv) w.y = -w.y;
      x = cadd(x, cmul(w, half[(R * r + q) * N + km]));
    }
    out[e] = x;
    if (out32) out32[e] = cx<float>{(float)x.x, (float)x.y};
  }
}

// dst = (float) src, elementwise over complex values.
__global__ void k_c64to32(const cx<double>* src, cx<float>* dst, size_t count) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = cx<float>{(float)src[e].x, (float)src[e].y};
}

// ---- power step (FP32) ----------------------------------------------------

struct SymPowerArgs {
  const uint32_t* hq;     // [B][n] (h << 2) | q
  const uint32_t* srt1;   // [B][n] sorted (h << 2) | q
  const uint32_t* ord1;   // [B][n]
  const uint32_t* srt2;   // [B][n] sorted (2h mod b << 2) | 2q mod 4
  const uint32_t* ord2;   // [B][n]
  int n, B;
  const cx<float>* S;     // [B][b] spectra
  const cx<float>* s;     // [B][b] time-domain sketches
  const cx<float>* tw;    // pass table of the b-point transform
  const cx<float>* tw2;   // pass table of the b/2-point transform
  const float* U;         // [L][n]
  float* V;               // [L][B][n]  Re v
  double* lam_per;        // [L][B] u . Re v (mode 1)
  int mode;
};

// Threads of the symmetric power kernel: 16 points per thread, at least 64.
constexpr int sym_threads(int logb) { return logb >= 10 ? (1 << (logb - 4)) : 64; }
// Dynamic LDS: the b-point sequence (split re/im, padded), u and the partial
// read-offs (n floats each).
constexpr size_t sym_power_lds(int logb, int n) {
  return align16(sizeof(float) * 2 * (size_t)padded_len(1 << logb)) + 2 * align16(sizeof(float) * (size_t)n);
}

template <int LOGB>
__global__ __launch_bounds__(sym_threads(LOGB)) void k_sym_power(SymPowerArgs a) {
  constexpr int b = 1 << LOGB;
  constexpr int NT = sym_threads(LOGB);
  constexpr int PL = padded_len(b);
  constexpr int PK = (b + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char lds[];
  float* re = reinterpret_cast<float*>(lds);
  const Soa<float> buf{re, re + PL};
  float* u = reinterpret_cast<float*>(lds + align16(sizeof(float) * 2 * (size_t)PL));
  float* vp = u + align16(sizeof(float) * (size_t)a.n) / sizeof(float);
  const int n = a.n, B = a.B;
  const int m = blockIdx.x, tau = blockIdx.y;
  const size_t tb = (size_t)m * n;
  const Twid<float> tw{a.tw, nullptr};
  for (int e = threadIdx.x; e < n; e += NT) {
    u[e] = a.U[(size_t)tau * n + e];
    vp[e] = 0.f;
  }
  // U_1 = F(s_u), kept in registers for the products
  for (int t = threadIdx.x; t < 2 * PL; t += NT) re[t] = 0.f;
  __syncthreads();
  auto put = [&](uint32_t t, cx<float> v) { buf.put((int)t, v); };
  sym_count_sketch<float>(a.srt1 + tb, a.ord1 + tb, n, NT, [&](uint32_t i) { return u[i]; }, put);
  __syncthreads();
  fft_soa<float, LOGB, NT, false>(buf, tw);
  cx<float> u1[PK];
#pragma unroll
  for (int q = 0; q < PK; ++q) {
    const int k = threadIdx.x + q * NT;
    u1[q] = k < b ? buf.get(k) : cx<float>{0.f, 0.f};
  }
  __syncthreads();
  // U_2 = F(s_2): s_2 sits on the even positions 2h mod b only, so U_2 is the
  // b/2-point transform E of its even samples, repeated: U_2[k] = E[k mod b/2]
  constexpr int H = b / 2;
  constexpr int PH = PK / 2;  // the thread's bins below b/2 (NT divides b/2)
  const Twid<float> tw2{a.tw2, nullptr};
  for (int t = threadIdx.x; t < 2 * PL; t += NT) re[t] = 0.f;
  __syncthreads();
  auto put2 = [&](uint32_t t, cx<float> v) { buf.put((int)(t >> 1), v); };
  sym_count_sketch<float>(a.srt2 + tb, a.ord2 + tb, n, NT, [&](uint32_t i) { return u[i] * u[i]; }, put2);
  __syncthreads();
  fft_soa<float, LOGB - 1, NT, false>(buf, tw2);
  // P_1 = S o (conj U_1^2 + conj U_2) in place at bins k and k + b/2, which
  // share E[k] (each thread writes only the position it read and one above
  // b/2); P_2 = S o conj U_1 kept
  const cx<float>* Sm = a.S + (size_t)m * b;
#pragma unroll
  for (int q = 0; q < PH; ++q) {
    const int k = threadIdx.x + q * NT;
    const cx<float> c2 = cconj(buf.get(k));
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int qq = q + half * PH, kk = k + half * H;
      const cx<float> sk = Sm[kk];
      const cx<float> c1 = cconj(u1[qq]);
      buf.put(kk, cmul(sk, cadd(cmul(c1, c1), c2)));
      u1[qq] = cmul(sk, c1);
    }
  }
  __syncthreads();
  // With n small against b both inverses leave out their last two passes and
  // the read-offs form the outputs they need from the groups before them.
  constexpr bool PR1 = output_from_groups_ok(b, NT) && LOGB < 14, PR2 = output_from_groups_ok(H, NT);
  constexpr int NS1 = pass_stride(b, NT, 1), NS2 = pass_stride(H, NT, 1);
  const bool prune1 = PR1 && n * pass_radix(b, NS1, fft_rmax(b, NT)) <= b;
  const bool prune2 = PR2 && n * pass_radix(H, NS2, fft_rmax(H, NT)) <= H;
  if constexpr (PR1) {
    fft_soa<float, LOGB, NT, true, true, 2>(buf, tw);
    if (!prune1) fft_soa_from<float, LOGB, NT, true, NS1, 0, true>(buf, tw);
  } else {
    fft_soa<float, LOGB, NT, true>(buf, tw);
  }
  const float sc = 1.f / (float)b;
  const uint32_t* hq = a.hq + tb;
  for (int i = threadIdx.x; i < n; i += NT) {
    const uint32_t e = hq[i];
    cx<float> c12;
    if constexpr (PR1) {
      c12 = prune1 ? inverse_output_from_groups<float, LOGB, NT>(buf, a.tw, (int)sym_pos(e))
                   : buf.get((int)sym_pos(e));
    } else {
      c12 = buf.get((int)sym_pos(e));
    }
    const cx<float> c = rot(c12, (4 - sym_rot(e)) & 3);  // conj(sigma) c12[h]
    vp[i] = c.x * (sc / 6.f);
  }
  __syncthreads();
  // c_3 is read at even positions only: c_3[2t] is the b/2-point inverse
  // transform of the folded spectrum P_2[k] + P_2[k + b/2]
#pragma unroll
  for (int q = 0; q < PH; ++q) buf.put(threadIdx.x + q * NT, cadd(u1[q], u1[q + PH]));
  __syncthreads();
  if constexpr (PR2) {
    fft_soa<float, LOGB - 1, NT, true, true, 2>(buf, tw2);
    if (!prune2) fft_soa_from<float, LOGB - 1, NT, true, NS2, 0, true>(buf, tw2);
  } else {
    fft_soa<float, LOGB - 1, NT, true>(buf, tw2);
  }
  const cx<float>* sm = a.s + (size_t)m * b;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const uint32_t e = hq[i];
    const uint32_t h = sym_pos(e);
    const int qq = sym_rot(e);
    const float ui = u[i];
    const int ph = (int)(h & (uint32_t)(H - 1));
    cx<float> c3e;
    if constexpr (PR2) {
      c3e = prune2 ? inverse_output_from_groups<float, LOGB - 1, NT>(buf, a.tw2, ph) : buf.get(ph);
    } else {
      c3e = buf.get(ph);
    }
    const cx<float> c3 = rot(c3e, (8 - 2 * qq) & 3);  // c_3[2h mod b]
    const cx<float> s3 = rot(sm[(3u * h) & (uint32_t)(b - 1)], (12 - 3 * qq) & 3);
    const float v = vp[i] + (ui * c3.x * sc + ui * ui * s3.x) * (1.f / 3.f);
    a.V[((size_t)tau * B + m) * n + i] = v;
    acc += (double)ui * (double)v;
  }
  if (a.mode == 1) {
    __shared__ double red[NT / 64];
    const double lam = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) a.lam_per[(size_t)tau * B + m] = lam;
  }
}

// ---- power step at b = R M, M = 16384 (FP32, split transforms) -------------
// At b = 32768 and 65536 the complex b-point sequence does not fit one
// work-group's LDS.  The step runs as three launches through a global buffer
// E of NR = R + R/2 rows of M complex values per (restart, sketch):
//   k_sym_split_fwd: row r < R is the M-point transform of the residue class r
//     mod R of s_u (its positions h / R); row R + r2 that of the residue class r2
//     mod R/2 of the even-position sketch s_2 halved (positions (2h mod b)/2);
//   k_sym_split_mid: per bin k < M, U_1 and U_2 at the R bins j = k + qM by
//     recombination, P_1 = S o (conj U_1^2 + conj U_2) and P_2 = S o conj U_1,
//     then the folds that the inverses need:
//       A_rho[k]   = sum_q W_b^{-rho (k + qM)} P_1[k + qM]           (rho < R),
//       A2_rho2[k] = sum_q' W_b^{-2 rho2 (k + q'M)} (P_2 + P_2[. + b/2])[k + q'M]  (rho2 < R/2),
//     written over the same rows;
//   k_sym_split_out: the R + R/2 inverse M-point transforms, one after the
//     other in LDS; c_12[R t + rho] = IFFT(A_rho)[t] / b and
//     c_3[2 ((R/2) t + rho2)] = IFFT(A2_rho2)[t] / b are read at h and at
//     2h mod b, and s at 3h mod b, into the read-off of the one-launch kernel.
constexpr int kSymSplitLogM = 14;

struct SymSplitArgs {
  const uint32_t* hq;     // [B][n] (h << 2) | q
  const uint32_t* srt1;   // [B][n] sorted (h << 2) | q
  const uint32_t* ord1;
  const uint32_t* srt2;   // [B][n] sorted (2h mod b << 2) | 2q mod 4
  const uint32_t* ord2;
  int n, B, b;
  const cx<float>* S;     // [B][b] spectra
  const cx<float>* s;     // [B][b] time-domain sketches
  const cx<float>* twM;   // pass table of the M-point transform
  const cx<float>* Wb;    // W_b^x, x < b
  const float* U;         // [L][n]
  cx<float>* E;           // [L][B][NR][M]
  float* V;               // [L][B][n]  Re v
  double* lam_per;        // [L][B] u . Re v (mode 1)
  int mode;
};

// LDS of the split forward and output kernels: the padded M-point sequence,
// then u and the partial read-offs (n floats each).
constexpr size_t sym_split_lds(int n) {
  return align16(sizeof(float) * 2 * (size_t)padded_len(1 << kSymSplitLogM)) + 2 * align16(sizeof(float) * (size_t)n);
}

template <int R>
__global__ __launch_bounds__(sym_threads(kSymSplitLogM)) void k_sym_split_fwd(SymSplitArgs a) {
  constexpr int LOGM = kSymSplitLogM, M = 1 << LOGM, NT = sym_threads(LOGM), PL = padded_len(M);
  constexpr int NR = R + R / 2;
  extern __shared__ __align__(16) unsigned char lds[];
  float* re = reinterpret_cast<float*>(lds);
  const Soa<float> buf{re, re + PL};
  float* u = reinterpret_cast<float*>(lds + align16(sizeof(float) * 2 * (size_t)PL));
  const int n = a.n, m = blockIdx.x, tau = blockIdx.y, row = blockIdx.z;
  const size_t tb = (size_t)m * n;
  for (int e = threadIdx.x; e < n; e += NT) u[e] = a.U[(size_t)tau * n + e];
  for (int t = threadIdx.x; t < 2 * PL; t += NT) re[t] = 0.f;
  __syncthreads();
  if (row < R) {
    sym_count_sketch<float>(a.srt1 + tb, a.ord1 + tb, n, NT, [&](uint32_t i) { return u[i]; },
                            [&](uint32_t t, cx<float> v) {
                              if ((int)(t & (uint32_t)(R - 1)) == row) buf.put((int)(t / R), v);
                            });
  } else {
    constexpr int R2 = R / 2;
    const int r2 = row - R;
    sym_count_sketch<float>(a.srt2 + tb, a.ord2 + tb, n, NT, [&](uint32_t i) { return u[i] * u[i]; },
                            [&](uint32_t t, cx<float> v) {
                              const uint32_t th = t >> 1;
                              if ((int)(th & (uint32_t)(R2 - 1)) == r2) buf.put((int)(th / R2), v);
                            });
  }
  __syncthreads();
  const Twid<float> tw{a.twM, nullptr};
  fft_soa<float, LOGM, NT, false>(buf, tw);
  cx<float>* dst = a.E + (((size_t)tau * a.B + m) * NR + row) * M;
  for (int k = threadIdx.x; k < M; k += NT) dst[k] = buf.get(k);
}

template <int R>
__global__ __launch_bounds__(256) void k_sym_split_mid(SymSplitArgs a) {
  constexpr int M = 1 << kSymSplitLogM, NR = R + R / 2, R2 = R / 2;
  const int m = blockIdx.x, tau = blockIdx.y;
  const int k = blockIdx.z * 256 + threadIdx.x;
  if (k >= M) return;
  const int b = a.b;
  const uint32_t bm = (uint32_t)b - 1u;
  cx<float>* Er = a.E + ((size_t)tau * a.B + m) * NR * M;
  auto W = [&](long x) { return a.Wb[(uint32_t)x & bm]; };
  cx<float> e[R], e2[R2];
#pragma unroll
  for (int r = 0; r < R; ++r) e[r] = Er[(size_t)r * M + k];
#pragma unroll
  for (int r = 0; r < R2; ++r) e2[r] = Er[(size_t)(R + r) * M + k];
  const cx<float>* Sm = a.S + (size_t)m * b;
  cx<float> P1[R], P2[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const long j = k + (long)q * M;
    cx<float> u1 = e[0];
#pragma unroll
    for (int r = 1; r < R; ++r) u1 = cadd(u1, cmul(W((long)r * j), e[r]));
    const long jp = k + (long)(q % R2) * M;  // j mod b/2
    cx<float> u2 = e2[0];
#pragma unroll
    for (int r = 1; r < R2; ++r) u2 = cadd(u2, cmul(W(2L * r * jp), e2[r]));
    const cx<float> sk = Sm[j];
    const cx<float> c1 = cconj(u1);
    P1[q] = cmul(sk, cadd(cmul(c1, c1), cconj(u2)));
    P2[q] = cmul(sk, c1);
  }
#pragma unroll
  for (int rho = 0; rho < R; ++rho) {
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < R; ++q)
      acc = cadd(acc, rho == 0 ? P1[q] : cmulc(P1[q], W((long)rho * (k + (long)q * M))));
    Er[(size_t)rho * M + k] = acc;
  }
#pragma unroll
  for (int r2 = 0; r2 < R2; ++r2) {
    cx<float> acc = {0.f, 0.f};
#pragma unroll
    for (int q = 0; q < R2; ++q) {
      const cx<float> f = cadd(P2[q], P2[q + R2]);
      acc = cadd(acc, r2 == 0 ? f : cmulc(f, W(2L * r2 * (k + (long)q * M))));
    }
    Er[(size_t)(R + r2) * M + k] = acc;
  }
}

template <int R>
__global__ __launch_bounds__(sym_threads(kSymSplitLogM)) void k_sym_split_out(SymSplitArgs a) {
  constexpr int LOGM = kSymSplitLogM, M = 1 << LOGM, NT = sym_threads(LOGM), PL = padded_len(M);
  constexpr int NR = R + R / 2, R2 = R / 2;
  extern __shared__ __align__(16) unsigned char lds[];
  float* re = reinterpret_cast<float*>(lds);
  const Soa<float> buf{re, re + PL};
  float* u = reinterpret_cast<float*>(lds + align16(sizeof(float) * 2 * (size_t)PL));
  float* vp = u + align16(sizeof(float) * (size_t)a.n) / sizeof(float);
  const int n = a.n, B = a.B, b = a.b, m = blockIdx.x, tau = blockIdx.y;
  const size_t tb = (size_t)m * n;
  const uint32_t* hq = a.hq + tb;
  const float sc = 1.f / (float)b;
  for (int e = threadIdx.x; e < n; e += NT) {
    u[e] = a.U[(size_t)tau * n + e];
    vp[e] = 0.f;
  }
  const Twid<float> tw{a.twM, nullptr};
  const cx<float>* Er = a.E + ((size_t)tau * B + m) * NR * M;
  for (int row = 0; row < NR; ++row) {
    __syncthreads();  // the previous row's readers of the buffer are done
    for (int k = threadIdx.x; k < M; k += NT) buf.put(k, Er[(size_t)row * M + k]);
    __syncthreads();
    fft_soa<float, LOGM, NT, true>(buf, tw);
    for (int i = threadIdx.x; i < n; i += NT) {
      const uint32_t e = hq[i];
      const uint32_t h = sym_pos(e);
      const int qq = sym_rot(e);
      if (row < R) {
        if ((int)(h & (uint32_t)(R - 1)) == row) {  // conj(sigma) c_12[h]
          const cx<float> c = rot(buf.get((int)(h / R)), (4 - qq) & 3);
          vp[i] += c.x * (sc / 6.f);
        }
      } else {
        const uint32_t t = h & (uint32_t)(b / 2 - 1);  // c_3 at 2h mod b = 2t
        if ((int)(t & (uint32_t)(R2 - 1)) == row - R) {
          const cx<float> c3 = rot(buf.get((int)(t / R2)), (8 - 2 * qq) & 3);
          vp[i] += u[i] * c3.x * sc * (1.f / 3.f);
        }
      }
    }
  }
  __syncthreads();
  const cx<float>* sm = a.s + (size_t)m * b;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const uint32_t e = hq[i];
    const uint32_t h = sym_pos(e);
    const int qq = sym_rot(e);
    const float ui = u[i];
    const cx<float> s3 = rot(sm[(3u * h) & (uint32_t)(b - 1)], (12 - 3 * qq) & 3);
    const float v = vp[i] + ui * ui * s3.x * (1.f / 3.f);
    a.V[((size_t)tau * B + m) * n + i] = v;
    acc += (double)ui * (double)v;
  }
  if (a.mode == 1) {
    __shared__ double red[NT / 64];
    const double lam = block_sum<NT>(acc, red);
    if (threadIdx.x == 0) a.lam_per[(size_t)tau * B + m] = lam;
  }
}

// ---- lambda_hat and deflation (FP64) ---------------------------------------

// cs[m][p-1] = the count sketch of u^p with sigma^p at p h mod b (p = 1, 2, 3),
// complex, for the run heads of the sorted tables; the rows are zero on entry.
// grid = (B, 3), 256 threads.
__global__ __launch_bounds__(256) void k_sym_cs64(const uint32_t* srt, const uint32_t* ord, int n, int b, int B,
                                                  const double* u, cx<double>* cs) {
  const int m = blockIdx.x, p = blockIdx.y + 1;
  const size_t tb = ((size_t)(p - 1) * B + m) * n;
  cx<double>* row = cs + ((size_t)m * 3 + (p - 1)) * b;
  sym_count_sketch<double>(srt + tb, ord + tb, n, 256,
                           [&](uint32_t i) { const double x = u[i]; return p == 1 ? x : (p == 2 ? x * x : x * x * x); },
                           [&](uint32_t t, cx<double> v) { row[t] = v; });
}

// Per sketch m: lam_per[m] = Re <s, s_X> = (1/b) Re sum_k S[k] conj(X[k]),
// X = U_1^3 / 6 + U_2 U_1 / 2 + U_3 / 3, and cube[m][k] = U_1[k]^3 (the
// spectrum of the full symmetric sketch of u^(x)3).  grid = B, 1024 threads.
__global__ __launch_bounds__(1024) void k_sym_lam(const cx<double>* S, const cx<double>* Uf, int b,
                                                  double* lam_per, cx<double>* cube) {
  __shared__ double red[16];
  const int m = blockIdx.x;
  const cx<double>* U1 = Uf + (size_t)m * 3 * b;
  const cx<double>* U2 = U1 + b;
  const cx<double>* U3 = U2 + b;
  double acc = 0.0;
  for (int k = threadIdx.x; k < b; k += 1024) {
    const cx<double> c3 = cmul(cmul(U1[k], U1[k]), U1[k]);
    const cx<double> x = cadd(cadd(cscale(c3, 1.0 / 6.0), cscale(cmul(U2[k], U1[k]), 0.5)),
                              cscale(U3[k], 1.0 / 3.0));
    const cx<double> sk = S[(size_t)m * b + k];
    acc += sk.x * x.x + sk.y * x.y;
    cube[(size_t)m * b + k] = c3;
  }
  const double s = block_sum<1024>(acc, red);
  if (threadIdx.x == 0) lam_per[m] = s / (double)b;
}

// X[e] -= lam * D[e] (complex), optional FP32 copy of X; scale applies to D.
__global__ void k_sym_axpy(cx<double>* X, cx<float>* X32, const cx<double>* D, const double* lam, double scale,
                           size_t count) {
  const double l = *lam * scale;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    const cx<double> x = csub(X[e], cscale(D[e], l));
    X[e] = x;
    if (X32) X32[e] = cx<float>{(float)x.x, (float)x.y};
  }
}

}  // namespace tsk
