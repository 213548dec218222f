// In-LDS FFT building blocks for gfx950 (wave64).
//
// One work-group transforms one sequence held in LDS.  Layout: real and
// imaginary parts in two separate arrays ("SoA"), element p stored at
// p + p/16, so that the stride-16 writes of a radix-16 pass and the
// unit-stride reads both hit distinct LDS banks.
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
// Twiddles: W_b^j = exp(-2 pi i j / b) = thi[j >> 6] * tlo[j & 63], with
// tlo[j] = W_b^j (j < 64) and thi[j] = W_b^(64 j) (j <= b/64), both in LDS and
// built on the host in FP64.  Within a butterfly the powers w^r are formed
// from w by multiplication (depth <= 4).  The inverse transform conjugates
// and carries no 1/N factor.
#pragma once

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

// Padded LDS position of element p.
__device__ __forceinline__ constexpr int pidx(int p) { return p + (p >> 4); }
// Words needed for an N-element padded array.
constexpr int padded_len(int n) { return n + (n >> 4) + 1; }

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
};

// Two-level twiddle table for base b in LDS.
template <typename R>
struct Twiddle {
  const cx<R>* tlo;  // [64]
  const cx<R>* thi;  // [b/64 + 1]
  __device__ __forceinline__ cx<R> w(int j) const { return cmul(thi[j >> 6], tlo[j & 63]); }
};

// Copies the global table (tlo[64] then thi[b/64+1]) into LDS `dst`; ends
// with a barrier, so the table is ready for every thread on return.
template <typename R>
__device__ __forceinline__ Twiddle<R> load_twiddles(cx<R>* dst, const cx<R>* __restrict__ src, int b,
                                                    int nt) {
  const int cnt = 64 + b / 64 + 1;
  for (int t = threadIdx.x; t < cnt; t += nt) dst[t] = src[t];
  __syncthreads();
  return Twiddle<R>{dst, dst + 64};
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

// v[r] *= w^r for r = 1..RAD-1.  Powers are formed on the fly from w, w^2,
// w^4 and w^8 (multiplication depth <= 4), so only those stay live.
template <typename R, int RAD>
__device__ __forceinline__ void apply_twiddles(cx<R>* v, cx<R> w) {
  v[1] = cmul(v[1], w);
  if constexpr (RAD > 2) {
    const cx<R> w2 = cmul(w, w);
    v[2] = cmul(v[2], w2);
    v[3] = cmul(v[3], cmul(w2, w));
    if constexpr (RAD > 4) {
      const cx<R> w4 = cmul(w2, w2);
      v[4] = cmul(v[4], w4);
      v[5] = cmul(v[5], cmul(w4, w));
      v[6] = cmul(v[6], cmul(w4, w2));
      v[7] = cmul(v[7], cmul(w4, cmul(w2, w)));
      if constexpr (RAD > 8) {
        const cx<R> w8 = cmul(w4, w4);
        v[8] = cmul(v[8], w8);
        v[9] = cmul(v[9], cmul(w8, w));
        v[10] = cmul(v[10], cmul(w8, w2));
        v[11] = cmul(v[11], cmul(w8, cmul(w2, w)));
        v[12] = cmul(v[12], cmul(w8, w4));
        v[13] = cmul(v[13], cmul(cmul(w8, w4), w));
        v[14] = cmul(v[14], cmul(cmul(w8, w4), w2));
        v[15] = cmul(v[15], cmul(cmul(w8, w4), cmul(w2, w)));
      }
    }
  }
}

// Offset, in padded positions, of element p + s from element p when s is r
// times a power-of-two stride S and p is aligned as in a Stockham pass (the
// group p .. p + (R-1) S never straddles a 16-block differently):
// pidx(p + r S) - pidx(p) = r S + (r S >> 4).
constexpr int poff(int rs) { return rs + (rs >> 4); }

// One Stockham pass over an N-point sequence with radix RAD and stride NS.
template <typename R, int N, int RAD, int NS, int NT, bool INV>
__device__ __forceinline__ void stockham_pass(const Soa<R>& buf, const Twiddle<R>& tw, int b) {
  constexpr int NB = N / RAD;
  constexpr int PER = (NB + NT - 1) / NT;
  // Opaque copy of the thread index: addresses are recomputed in every pass
  // instead of being hoisted and kept live across the whole kernel.
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
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
        const int k = j & (NS - 1);
        cx<R> w = tw.w(k * (b / (NS * RAD)));
        if (INV) w.y = -w.y;
        apply_twiddles<R, RAD>(v[q], w);
      }
      dft_r<R, RAD, INV>(v[q]);
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

template <typename R, int N, int NS, int NT, int RMAX, bool INV>
__device__ __forceinline__ void fft_passes(const Soa<R>& buf, const Twiddle<R>& tw, int b) {
  if constexpr (NS < N) {
    constexpr int REM = N / NS;
    constexpr int RAD = REM >= RMAX ? RMAX : REM;
    stockham_pass<R, N, RAD, NS, NT, INV>(buf, tw, b);
    fft_passes<R, N, NS * RAD, NT, RMAX, INV>(buf, tw, b);
  }
}

// Complex FFT of length N = 2^LOGN in LDS (SoA, padded); ends with a barrier.
// The radix is N/NT (each thread one butterfly per pass), at most 16.
template <typename R, int LOGN, int NT, bool INV>
__device__ __forceinline__ void fft_soa(const Soa<R>& buf, const Twiddle<R>& tw, int b) {
  constexpr int PERT = (1 << LOGN) / NT;
  constexpr int RMAX = PERT >= 16 ? 16 : (PERT >= 8 ? 8 : (PERT >= 4 ? 4 : 2));
  fft_passes<R, (1 << LOGN), 1, NT, RMAX, INV>(buf, tw, b);
}

}  // namespace tsk
