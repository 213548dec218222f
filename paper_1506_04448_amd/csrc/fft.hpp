// In-LDS batched FFT building blocks for gfx950 (wave64).
//
// One work-group transforms one sequence held in LDS.  The transform is the
// Stockham auto-sort formulation: each pass reads R inputs at stride N/R,
// applies the twiddles of the current sub-transform, does a radix-R DFT in
// registers and writes the R outputs at stride Ns, so the result comes out in
// natural order without a bit-reversal pass.  Every pass keeps all of its
// inputs in registers between one barrier and the next, which makes a single
// LDS buffer enough (the write of one pass may overwrite what another thread
// has already read).
//
// Twiddles come from a table tw[j] = exp(-2 pi i j / NTW), NTW = 2^logNtw >= N,
// built on the host in FP64 and rounded once to the working type; the inverse
// transform uses their conjugates and carries no 1/N factor.
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

// Twiddle w = tw[idx], conjugated for the inverse transform.
template <typename R, bool INV>
__device__ __forceinline__ cx<R> twiddle(const cx<R>* __restrict__ tw, int idx) {
  cx<R> w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// Radix-4 DFT in registers: y_q = sum_r x_r W4^{rq}, W4 = -i (forward) or +i.
template <typename R, bool INV>
__device__ __forceinline__ void dft4(cx<R>& v0, cx<R>& v1, cx<R>& v2, cx<R>& v3) {
  cx<R> a = cadd(v0, v2), b = csub(v0, v2), c = cadd(v1, v3), d = csub(v1, v3);
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

// Complex FFT of length N = 2^LOGN held in LDS `buf`, NT threads.
// Radix-4 passes, plus one radix-2 pass when LOGN is odd.
// Ends with a barrier, so the result is visible to the whole work-group.
template <typename R, int LOGN, int NT, bool INV>
__device__ void fft_lds(cx<R>* buf, const cx<R>* __restrict__ tw, int logNtw) {
  constexpr int N = 1 << LOGN;
  constexpr int NB4 = N / 4;
  constexpr int PER = (NB4 + NT - 1) / NT;
  const int tid = threadIdx.x;
  int logNs = 0;
#pragma unroll 1
  for (int p = 0; p < LOGN / 2; ++p) {
    const int Ns = 1 << logNs;
    const int sh = logNtw - logNs - 2;
    cx<R> v[PER][4];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB4 % NT) == 0 || j < NB4) {
        const int k = j & (Ns - 1);
        v[q][0] = buf[j];
        v[q][1] = buf[j + NB4];
        v[q][2] = buf[j + 2 * NB4];
        v[q][3] = buf[j + 3 * NB4];
        if (logNs > 0) {
          v[q][1] = cmul(v[q][1], twiddle<R, INV>(tw, k << sh));
          v[q][2] = cmul(v[q][2], twiddle<R, INV>(tw, (2 * k) << sh));
          v[q][3] = cmul(v[q][3], twiddle<R, INV>(tw, (3 * k) << sh));
        }
        dft4<R, INV>(v[q][0], v[q][1], v[q][2], v[q][3]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = tid + q * NT;
      if ((NB4 % NT) == 0 || j < NB4) {
        const int k = j & (Ns - 1);
        const int d = ((j - k) << 2) + k;
        buf[d] = v[q][0];
        buf[d + Ns] = v[q][1];
        buf[d + 2 * Ns] = v[q][2];
        buf[d + 3 * Ns] = v[q][3];
      }
    }
    __syncthreads();
    logNs += 2;
  }
  if (LOGN & 1) {
    // Final radix-2 pass, Ns = N/2: butterfly j reads and writes j and j+N/2.
    constexpr int NB2 = N / 2;
    const int sh = logNtw - LOGN;
    for (int j = tid; j < NB2; j += NT) {
      cx<R> a = buf[j];
      cx<R> b = cmul(buf[j + NB2], twiddle<R, INV>(tw, j << sh));
      buf[j] = cadd(a, b);
      buf[j + NB2] = csub(a, b);
    }
    __syncthreads();
  }
}

}  // namespace tsk
