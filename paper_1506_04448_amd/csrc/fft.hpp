// In-LDS FFT building blocks for gfx950 (wave64).
//
// One work-group transforms one sequence held in LDS.  Layout: real and
// imaginary parts in two separate arrays ("SoA"), element p stored at
// p + 5 (p / 64) (see pidx), which keeps the passes' strided accesses on
// distinct LDS banks.
//
// The transform is the Stockham auto-sort formulation: each pass reads R
// inputs at stride N/R, applies the twiddles of the current sub-transform,
// does a radix-R DFT in registers and writes the R outputs at stride Ns, so
// the result comes out in natural order without a bit-reversal pass.  All of
// a pass's inputs are held in registers between two barriers, so one LDS
// buffer suffices.  The radix is the number of points per thread (at most 16)
// and a last smaller pass takes the remaining bits; every pass is unrolled at
// compile time.
//
// Twiddles come from per-pass tables in global memory (see pass_table_len),
// read straight into the butterfly; the inverse transform conjugates them and
// carries no 1/N factor.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

namespace tsk {

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cscale(cx<R> a, R s) { return {a.x * s, a.y * s}; }

// Padded LDS position of element p: five spare words after every 64.  With
// 64 four-byte banks this keeps the unit-stride reads and the stride-1, 8,
// 64 ... writes of the radix-8 Stockham passes (nearly) free of bank
// conflicts, and the position of p + s is pidx(p) + poff(s) for every access
// the passes make, so offsets fold into the instructions.
__device__ __forceinline__ constexpr int pidx(int p) {
  // at run time a 24-bit multiply-add (full rate) rather than the 64-bit
  // multiply-add the compiler otherwise picks for p + 5 (p >> 6)
  return __builtin_is_constant_evaluated() ? p + 5 * (p >> 6)
                                           : p + (int)__umul24((unsigned)(p >> 6), 5u);
}
// Words needed for an N-element padded array.
constexpr int padded_len(int n) { return n + 5 * (n >> 6) + 6; }

// Split-array view of a complex sequence in LDS.
template <typename R>
struct Soa {
  R* re;
  R* im;
  __device__ __forceinline__ cx<R> get(int p) const {
    const int q = pidx(p);
    return {re[q], im[q]};
  }
  __device__ __forceinline__ void put(int p, cx<R> v) const {
    const int q = pidx(p);
    re[q] = v.x;
    im[q] = v.y;
  }
  // by padded position
  __device__ __forceinline__ cx<R> at(int q) const { return {re[q], im[q]}; }
  __device__ __forceinline__ void put_at(int q, cx<R> v) const {
    re[q] = v.x;
    im[q] = v.y;
  }
};

// ---- twiddle tables ---------------------------------------------------------
// Radix plan of an N-point transform run by NT threads: every pass uses
// R = min(N/NT, 16) points per butterfly (a last pass takes what is left).
constexpr int fft_rmax(int N, int NT) {
  return (N / NT) >= 16 ? 16 : ((N / NT) >= 8 ? 8 : ((N / NT) >= 4 ? 4 : 2));
}
constexpr int pass_radix(int N, int NS, int RMAX) { return (N / NS) >= RMAX ? RMAX : N / NS; }
// Number of passes of the plan from stride NS on.
constexpr int passes_from(int N, int NS, int RMAX) {
  int c = 0;
  for (int ns = NS; ns < N; ns *= pass_radix(N, ns, RMAX)) ++c;
  return c;
}
// Stride of the pass that has `left` passes after it (0: the last pass).
constexpr int pass_stride(int N, int NT, int left) {
  int ns = 1;
  while (passes_from(N, ns, fft_rmax(N, NT)) > left + 1) ns *= pass_radix(N, ns, fft_rmax(N, NT));
  return ns;
}

// Per-pass twiddle table: for every pass with stride NS > 1 and radix R, the
// entries W_{NS R}^{r k} for r = 1..R-1 and k < NS, stored at
// [pass offset + (r-1) NS + k], so the lanes of a wave read consecutive
// entries.  Built on the host in FP64 and rounded once.  pass_table_off is
// the offset of the pass with stride NS.
constexpr int pass_table_off(int N, int NT, int NS) {
  int len = 0;
  for (int ns = 1; ns < NS;) {
    const int rad = pass_radix(N, ns, fft_rmax(N, NT));
    if (ns > 1) len += (rad - 1) * ns;
    ns *= rad;
  }
  return len;
}
constexpr int pass_table_len(int N, int NT) { return pass_table_off(N, NT, N); }

// Twiddles of one real transform of length b = 2H through an H-point complex
// transform: the pass table of the H-point FFT followed by W_b^k, k = 0..H.
template <typename R>
struct Twid {
  const cx<R>* pass;  // per-pass table (global)
  const cx<R>* wk;    // W_b^k (global)
  __device__ __forceinline__ cx<R> w(int k) const { return wk[k]; }
};

// Buffer-resource load of one complex twiddle: `voff` (per lane) and `soff`
// (uniform) are byte offsets from the resource's base.  All twiddles of a
// pass share one per-lane offset; the per-r row offsets go to scalar
// registers.  Out-of-range reads return zero.
constexpr unsigned kBufferWord3 = 0x00020000u;  // raw 32-bit buffer, gfx9 family
template <typename R>
__device__ __forceinline__ cx<R> tw_load(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
  if constexpr (sizeof(R) == 4) {
    return __builtin_bit_cast(cx<R>, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  } else {
    return __builtin_bit_cast(cx<R>, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  }
}

constexpr int twid_len(int H, int NT) { return pass_table_len(H, NT) + H + 1; }

// Radix of the last pass of the plan (the passes use fft_rmax, the last one
// takes the remaining factor).
constexpr int fft_last_radix(int N, int NT) {
  int rad = 2;
  for (int ns = 1; ns < N;) {
    rad = pass_radix(N, ns, fft_rmax(N, NT));
    ns *= rad;
  }
  return rad;
}

// ---- radix-R DFTs in registers (y_q = sum_r x_r W_R^{rq}, W_R = e^{-+2 pi i/R}) ----

template <typename R, bool INV>
__device__ __forceinline__ void dft2(cx<R>& a, cx<R>& b) {
  const cx<R> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cx<R>& v0, cx<R>& v1, cx<R>& v2, cx<R>& v3) {
  const cx<R> a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = csub(v1, v3);
  v0 = cadd(a, c);
  v2 = csub(a, c);
  if (!INV) {
    v1 = {b.x + d.y, b.y - d.x};  // b - i d
    v3 = {b.x - d.y, b.y + d.x};  // b + i d
  } else {
    v1 = {b.x - d.y, b.y + d.x};
    v3 = {b.x + d.y, b.y - d.x};
  }
}

// Multiply by W_8^e (e = 1, 2, 3) for the forward sign, conjugate for INV.
template <typename R, bool INV, int E>
__device__ __forceinline__ cx<R> rot8(cx<R> a) {
  constexpr R h = R(0.70710678118654752440084436210485);
  if (E == 0) return a;
  if (E == 2) return INV ? cx<R>{-a.y, a.x} : cx<R>{a.y, -a.x};
  if (E == 1) return INV ? cx<R>{h * (a.x - a.y), h * (a.x + a.y)} : cx<R>{h * (a.x + a.y), h * (a.y - a.x)};
  // E == 3: W8^3 = (-h, -h) forward
  return INV ? cx<R>{-h * (a.x + a.y), h * (a.x - a.y)} : cx<R>{h * (a.y - a.x), -h * (a.x + a.y)};
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cx<R>* x) {
  // 8 = 2 x 4: DFT4 over even/odd, twiddle by W8^{n2 k1}, DFT2.
  dft4<R, INV>(x[0], x[2], x[4], x[6]);
  dft4<R, INV>(x[1], x[3], x[5], x[7]);
  x[3] = rot8<R, INV, 1>(x[3]);
  x[5] = rot8<R, INV, 2>(x[5]);
  x[7] = rot8<R, INV, 3>(x[7]);
  cx<R> y[8];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<R> a = x[2 * k1], b = x[2 * k1 + 1];
    dft2<R, INV>(a, b);
    y[k1] = a;
    y[k1 + 4] = b;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = y[i];
}

// W_16^e for e in [0, 16): compile-time constants.
template <typename R, bool INV>
__device__ __forceinline__ cx<R> w16(int e) {
  constexpr R c1 = R(0.92387953251128675612818318939679);
  constexpr R s1 = R(0.38268343236508977172845998403040);
  constexpr R h = R(0.70710678118654752440084436210485);
  // forward W16^e = cos(2 pi e/16) - i sin(2 pi e/16)
  R c, s;
  switch (e & 15) {
    case 0: c = 1; s = 0; break;
    case 1: c = c1; s = s1; break;
    case 2: c = h; s = h; break;
    case 3: c = s1; s = c1; break;
    case 4: c = 0; s = 1; break;
    case 5: c = -s1; s = c1; break;
    case 6: c = -h; s = h; break;
    case 7: c = -c1; s = s1; break;
    case 8: c = -1; s = 0; break;
    case 9: c = -c1; s = -s1; break;
    case 10: c = -h; s = -h; break;
    case 11: c = -s1; s = -c1; break;
    case 12: c = 0; s = -1; break;
    case 13: c = s1; s = -c1; break;
    case 14: c = h; s = -h; break;
    default: c = c1; s = -s1; break;
  }
  return INV ? cx<R>{c, s} : cx<R>{c, -s};
}

template <typename R, bool INV>
__device__ __forceinline__ void dft16(cx<R>* x) {
  // 16 = 4 x 4: for each n2, DFT4 over x[n2 + 4 n1]; twiddle W16^{n2 k1};
  // then for each k1, DFT4 over n2; output index k1 + 4 k2.
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<R, INV>(x[n2], x[n2 + 4], x[n2 + 8], x[n2 + 12]);
#pragma unroll
  for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
    for (int k1 = 1; k1 < 4; ++k1) x[n2 + 4 * k1] = cmul(x[n2 + 4 * k1], w16<R, INV>(n2 * k1));
  cx<R> y[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<R> a = x[4 * k1], b = x[4 * k1 + 1], c = x[4 * k1 + 2], d = x[4 * k1 + 3];
    dft4<R, INV>(a, b, c, d);
    y[k1] = a;
    y[k1 + 4] = b;
    y[k1 + 8] = c;
    y[k1 + 12] = d;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) x[i] = y[i];
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft_r(cx<R>* x) {
  if constexpr (RAD == 2) dft2<R, INV>(x[0], x[1]);
  else if constexpr (RAD == 4) dft4<R, INV>(x[0], x[1], x[2], x[3]);
  else if constexpr (RAD == 8) dft8<R, INV>(x);
  else dft16<R, INV>(x);
}

// Offset, in padded positions, of element p + s from element p for the
// accesses of a Stockham pass (s = r times the pass's power-of-two stride, p
// aligned as the pass aligns it): pidx(p + s) - pidx(p) = s + 5 (s >> 6).
constexpr int poff(int rs) { return rs + 5 * (rs >> 6); }

// Twiddles of one pass held in registers: w[q][r-1] for the thread's q-th
// butterfly.  Loaded one pass ahead so the global loads overlap the previous
// pass's arithmetic.
template <typename R, int PER, int NR>
struct PassTw {
  cx<R> w[PER][NR > 0 ? NR : 1];
};

template <typename R, int N, int RAD, int NS, int NT, int TOFF>
__device__ __forceinline__ void load_pass_tw(PassTw<R, (N / RAD + NT - 1) / NT, RAD - 1>& t,
                                             const Twid<R>& tw, int tid) {
  constexpr int NB = N / RAD;
  constexpr int PER = (NB + NT - 1) / NT;
  if constexpr (NS > 1) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<cx<R>*>(tw.pass), 0, (TOFF + (RAD - 1) * NS) * (int)sizeof(cx<R>), kBufferWord3);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB % NT) == 0 || j < NB) {
        const unsigned voff = (unsigned)(j & (NS - 1)) * (unsigned)sizeof(cx<R>);
#pragma unroll
        for (int r = 1; r < RAD; ++r)
          t.w[q][r - 1] = tw_load<R>(rs, voff, (unsigned)((TOFF + (r - 1) * NS) * sizeof(cx<R>)));
      }
    }
  }
}

// One Stockham pass over an N-point sequence with radix RAD and stride NS,
// using the twiddles `t` loaded for it.
template <typename R, int N, int RAD, int NS, int NT, bool INV>
__device__ __forceinline__ void stockham_pass(const Soa<R>& buf,
                                              const PassTw<R, (N / RAD + NT - 1) / NT, RAD - 1>& t,
                                              int tid) {
  constexpr int NB = N / RAD;
  constexpr int PER = (NB + NT - 1) / NT;
  cx<R> v[PER][RAD];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    if ((NB % NT) == 0 || j < NB) {
      const int base = pidx(j);
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        v[q][r].x = buf.re[base + poff(r * NB)];
        v[q][r].y = buf.im[base + poff(r * NB)];
      }
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < RAD; ++r) {
          cx<R> w = t.w[q][r - 1];
          if (INV) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dft_r<R, RAD, INV>(v[q]);
      // Keep the butterfly ahead of the barrier: waves that have their
      // inputs compute while the others still read.
#pragma unroll
      for (int r = 0; r < RAD; ++r) asm volatile("" : "+v"(v[q][r].x), "+v"(v[q][r].y));
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int j = tid + q * NT;
    if ((NB % NT) == 0 || j < NB) {
      const int k = j & (NS - 1);
      const int base = pidx((j - k) * RAD + k);
#pragma unroll
      for (int r = 0; r < RAD; ++r) {
        buf.re[base + poff(r * NS)] = v[q][r].x;
        buf.im[base + poff(r * NS)] = v[q][r].y;
      }
    }
  }
  __syncthreads();
}

// Passes from stride NS on; `cur` holds this pass's twiddles.  With PF the
// next pass's twiddles are loaded before the current pass runs (their global
// loads overlap its arithmetic, at the cost of registers); without PF each
// pass loads its own at its start.
template <typename R, int N, int NS, int NT, int RMAX, bool INV, int TOFF, bool PF, int SKIP = 0>
__device__ __forceinline__ void fft_passes(
    const Soa<R>& buf, const Twid<R>& twp,
    const PassTw<R, (N / pass_radix(N, NS, RMAX) + NT - 1) / NT, pass_radix(N, NS, RMAX) - 1>& cur) {
  constexpr int RAD = pass_radix(N, NS, RMAX);
  constexpr int NS2 = NS * RAD;
  constexpr int TOFF2 = TOFF + (NS > 1 ? (RAD - 1) * NS : 0);
  // Opaque copy of the thread index: addresses are recomputed in every pass
  // instead of being hoisted and kept live across the whole kernel.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  constexpr int RAD2 = NS2 < N ? pass_radix(N, NS2, RMAX) : 2;
  PassTw<R, (N / RAD2 + NT - 1) / NT, RAD2 - 1> nxt;
  if constexpr (PF) {
    if constexpr (NS2 < N) load_pass_tw<R, N, RAD2, NS2, NT, TOFF2>(nxt, twp, tid);
    stockham_pass<R, N, RAD, NS, NT, INV>(buf, cur, tid);
  } else {
    PassTw<R, (N / RAD + NT - 1) / NT, RAD - 1> own;
    load_pass_tw<R, N, RAD, NS, NT, TOFF>(own, twp, tid);
    stockham_pass<R, N, RAD, NS, NT, INV>(buf, own, tid);
  }
  // SKIP: the last SKIP passes are left out (their inputs stay in the buffer).
  if constexpr (NS2 < N && passes_from(N, NS2, RMAX) > SKIP)
    fft_passes<R, N, NS2, NT, RMAX, INV, TOFF2, PF, SKIP>(buf, twp, nxt);
}

// Complex FFT of length N = 2^LOGN in LDS (SoA, padded); ends with a barrier.
// PF as in fft_passes.  SKIP = 1 leaves the last pass out: for a last
// pass of radix 2 the buffer then holds a[j] and b[j] = in[j + N/2], and
// X[j] = a[j] + W_N^j b[j], X[j + N/2] = a[j] - W_N^j b[j] (conjugate twiddle
// for INV), with W_N^j at pass_table_len(N, NT) - N/2 + j of the pass table.
template <typename R, int LOGN, int NT, bool INV, bool PF = true, int SKIP = 0>
__device__ __forceinline__ void fft_soa(const Soa<R>& buf, const Twid<R>& tw) {
  constexpr int N = 1 << LOGN;
  constexpr int RMAX = fft_rmax(N, NT);
  constexpr int RAD = pass_radix(N, 1, RMAX);
  static_assert(passes_from(N, 1, RMAX) > SKIP, "at least one pass runs");
  PassTw<R, (N / RAD + NT - 1) / NT, RAD - 1> first;  // the first pass has no twiddles
  fft_passes<R, N, 1, NT, RMAX, INV, 0, PF, SKIP>(buf, tw, first);
}

// The passes of the same transform from stride NS on (NS > 1), leaving the
// last SKIP out; ends with a barrier.  PF as in fft_passes.
template <typename R, int LOGN, int NT, bool INV, int NS, int SKIP = 0, bool PF = false>
__device__ __forceinline__ void fft_soa_from(const Soa<R>& buf, const Twid<R>& tw) {
  constexpr int N = 1 << LOGN;
  constexpr int RMAX = fft_rmax(N, NT);
  constexpr int RAD = pass_radix(N, NS, RMAX);
  constexpr int TOFF = pass_table_off(N, NT, NS);
  static_assert(NS > 1 && passes_from(N, NS, RMAX) > SKIP, "at least one twiddled pass runs");
  PassTw<R, (N / RAD + NT - 1) / NT, RAD - 1> cur;  // read only with PF
  if constexpr (PF) load_pass_tw<R, N, RAD, NS, NT, TOFF>(cur, tw, (int)threadIdx.x);
  fft_passes<R, N, NS, NT, RMAX, INV, TOFF, PF, SKIP>(buf, tw, cur);
}

// Whether inverse_output_from_groups applies to the plan of an N-point
// transform run by NT threads: at least three passes, the last of radix 2 or 4.
constexpr bool output_from_groups_ok(int N, int NT) {
  return passes_from(N, 1, fft_rmax(N, NT)) >= 3 && (fft_last_radix(N, NT) == 2 || fft_last_radix(N, NT) == 4);
}

// Output p of an inverse N-point transform run without its last two passes
// (fft_soa with SKIP = 2).  Before those passes group g < G = N / NS3 of the
// buffer holds the NS3-point transform D_g of the inputs congruent to g
// modulo G (D_g[k] at g NS3 + k), so z[p] = sum_g W_N^{-g p} D_g[p mod NS3].
// The sum is a Horner scheme in base 4 (base 2 at the top when G is not a
// power of 4) whose level l uses W_N^{-4^l p}, each read from the last
// pass's twiddle row (W_N^j, j < NSL) times a power of W_RL, so every term
// passes through a few roundings per level only.  `pass` is the pass table.
template <typename R, int LOGN, int NT>
__device__ __forceinline__ cx<R> inverse_output_from_groups(const Soa<R>& buf, const cx<R>* pass, int p) {
  constexpr int N = 1 << LOGN;
  static_assert(output_from_groups_ok(N, NT), "three passes or more, the last of radix 2 or 4");
  constexpr int NS3 = pass_stride(N, NT, 1);
  constexpr int NSL = pass_stride(N, NT, 0);
  constexpr int RL = N / NSL;
  constexpr int G = N / NS3;
  const cx<R>* wrow = pass + pass_table_off(N, NT, NSL);  // W_N^j, j < NSL
  // W_N^{-j} for any j: the row entry of j mod NSL times W_RL^{-(j / NSL)}.
  auto wneg = [&](int j) -> cx<R> {
    const cx<R> t = wrow[j & (NSL - 1)];
    const int q = (j / NSL) & (RL - 1);
    cx<R> w{t.x, -t.y};  // conj
    if constexpr (RL == 2) {
      if (q) w = {-w.x, -w.y};
    } else {  // times i^q
      if (q & 1) w = {-w.y, w.x};
      if (q & 2) w = {-w.x, -w.y};
    }
    return w;
  };
  auto mad = [](cx<R> x, cx<R> w, cx<R> y) -> cx<R> {
    return {x.x * w.x - x.y * w.y + y.x, x.x * w.y + x.y * w.x + y.y};
  };
  const int k = p & (NS3 - 1);
  const int pk = pidx(k);
  auto d = [&](int g) -> cx<R> {
    return buf.at(NS3 % 64 == 0 ? pk + poff(g * NS3) : pidx(g * NS3 + k));
  };
  constexpr int L4 = [] { int l = 0; for (int g = G; g >= 4; g /= 4) ++l; return l; }();  // levels of 4
  constexpr bool TOP2 = (1 << (2 * L4)) != G;  // one more level of 2
  cx<R> wl[L4 + 1];
#pragma unroll
  for (int l = 0; l < L4 + (TOP2 ? 1 : 0); ++l) wl[l] = wneg((int)(((unsigned)p << (2 * l)) & (unsigned)(N - 1)));
  // sum_{j < 4^(LVL+1)} w^j d(base + j), with wl[LVL] = w^(4^LVL)
  auto level = [&](auto&& self, auto lvl, int base) -> cx<R> {
    constexpr int LVL = decltype(lvl)::value;
    cx<R> acc;
#pragma unroll
    for (int c = 3; c >= 0; --c) {
      cx<R> x;
      if constexpr (LVL == 0)
        x = d(base + c);
      else
        x = self(self, std::integral_constant<int, LVL - 1>{}, base + c * (1 << (2 * LVL)));
      acc = c == 3 ? x : mad(acc, wl[LVL], x);
    }
    return acc;
  };
  if constexpr (!TOP2) {
    return level(level, std::integral_constant<int, L4 - 1>{}, 0);
  } else {
    constexpr int HALF = G / 2;
    cx<R> lo, hi;
    if constexpr (L4 == 0) {
      lo = d(0);
      hi = d(1);
    } else {
      lo = level(level, std::integral_constant<int, L4 - 1>{}, 0);
      hi = level(level, std::integral_constant<int, L4 - 1>{}, HALF);
    }
    return mad(hi, wl[L4], lo);  // wl[L4] = w^(4^L4) = w^HALF
  }
}

}  // namespace tsk
