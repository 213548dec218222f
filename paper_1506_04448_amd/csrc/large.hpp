// Transforms longer than one work-group's LDS holds (b = 32768 and 65536 in
// FP64, b = 65536 in FP32): the half-length sequence z (H = b/2 complex values)
// is split by residue, z_r[s] = z[R s + r], into R sub-sequences of length
// M = H / R that fit LDS; each is transformed in LDS by its own work-group and
// the length-H transform is recombined in global memory:
//   Z[k] = sum_r W_H^(r k) E_r[k mod M],          E_r = FFT_M(z_r)
// and, for the inverse, z_r = IFFT_M(A_r) with
//   A_r[k'] = W_H^(-r k') sum_q Y[k' + q M] W_R^(-r q).
// Every twiddle comes from one table of W_b^x, x in [0, b) (W_H^x = W_b^(2x)).
#pragma once

#include "kernels.hpp"

namespace tsk {

// W_b^x for any integer x (b a power of two: x mod b is x & (b - 1))
template <typename R>
__device__ __forceinline__ cx<R> wfull(const cx<R>* Wb, int b, long long x) {
  return Wb[(int)(x & (long long)(b - 1))];
}

// Forward sub-transforms of count sketches restricted to one residue class of
// the packed positions: grid (B, nvec, nmodes * R); block z = jj * R + r.
//   E[((vec * B + m) * nmodes + jj) * R + r][k], k < M
// The count sketch of vector `vec` uses the table rows of mode modes[jj].
template <typename R, typename UIn>
struct SubCsArgs {
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B, Rr, nmodes;
  int mode[3];
  const UIn* U;        // [nvec][n]
  const UIn* U2;       // [nvec][n] or null: the vector of the second mode (two-vector contraction)
  const cx<R>* twM;    // pass table of the M-point transform
  cx<R>* E;
};

template <typename R, int LOGM, typename UIn>
__global__ __launch_bounds__(threads_for_h<R>(LOGM)) void k_sub_cs(SubCsArgs<R, UIn> a) {
  constexpr int M = 1 << LOGM;
  constexpr int NT = threads_for_h<R>(LOGM);
  constexpr int PL = padded_len(M);
  __shared__ __align__(16) R re[2 * PL];
  R* im = re + PL;
  const Soa<R> buf{re, im};
  const int m = blockIdx.x, vec = blockIdx.y;
  const int jj = blockIdx.z / a.Rr, r = blockIdx.z % a.Rr;
  const int n = a.n;
  const size_t tb = ((size_t)m * 3 + a.mode[jj]) * n;
  const UIn* u = (jj == 1 && a.U2 ? a.U2 : a.U) + (size_t)vec * n;
  const unsigned Rr = (unsigned)a.Rr;
  for (int t = threadIdx.x; t < 2 * PL; t += NT) re[t] = R(0);
  __syncthreads();
  auto getu = [&](uint32_t i) -> R { return (R)u[i]; };
  auto store = [&](uint32_t t, R v) {
    const unsigned p = t >> 1;
    if (p % Rr == (unsigned)r) {
      const int q = pidx((int)(p / Rr));
      if (t & 1u) im[q] = v;
      else re[q] = v;
    }
  };
  count_sketch<R>(a.hxs + tb, a.ord + tb, n, NT, getu, store);
  __syncthreads();
  const Twid<R> tw{a.twM, nullptr};
  fft_soa<R, LOGM, NT, false>(buf, tw);
  cx<R>* out = a.E + ((((size_t)vec * a.B + m) * a.nmodes + jj) * a.Rr + r) * M;
  for (int k = threadIdx.x; k < M; k += NT) out[k] = buf.get(k);
}

// Z[k] = sum_r W_H^(r k) E_r[k mod M] for the sub-transforms E[r][M].
template <typename R>
__device__ __forceinline__ cx<R> recombine(const cx<R>* E, int M, int Rr, const cx<R>* Wb, int b, int k) {
  const int km = k % M;
  cx<R> z = E[km];
  for (int r = 1; r < Rr; ++r) z = cadd(z, cmul(wfull(Wb, b, 2LL * r * k), E[(size_t)r * M + km]));
  return z;
}

// FP64 rank-1 spectra from the sub-transforms of the three modes:
//   prod[vec][m][k] = prod_j X_j[k], k = 0..H,  X_j = r2c post-processing of Z_j;
//   lam_per[vec][m] = <s^(m), s^(m)(u_vec^(x)3)> by Parseval when S64 != null.
// grid (B, nvec), 1024 threads.
__global__ __launch_bounds__(1024) void k_combine_rank1(const cx<double>* E, int B, int b, int M, int Rr,
                                                        const cx<double>* Wb, const cx<double>* S64,
                                                        cx<double>* prod, double* lam_per) {
  __shared__ double red[16];
  const int m = blockIdx.x, vec = blockIdx.y;
  const int H = b / 2;
  const cx<double>* Ev = E + (((size_t)vec * B + m) * 3) * Rr * (size_t)M;
  cx<double>* out = prod + ((size_t)vec * B + m) * (H + 1);
  const cx<double>* S = S64 ? S64 + (size_t)m * (H + 1) : nullptr;
  double acc = 0.0;
  // one thread per bin pair (k, H - k), k <= H/2: both bins use the same two
  // recombined values of each mode
  for (int k = threadIdx.x; k <= H / 2; k += 1024) {
    const int kh = H - k;
    cx<double> p = {1.0, 0.0}, ph = {1.0, 0.0};
    for (int j = 0; j < 3; ++j) {
      const cx<double>* Ej = Ev + (size_t)j * Rr * M;
      const cx<double> Za = recombine(Ej, M, Rr, Wb, b, k);
      const cx<double> Zb = recombine(Ej, M, Rr, Wb, b, kh % H);
      p = cmul(p, r2c_post(Za, Zb, Wb[k]));
      ph = cmul(ph, r2c_post(Zb, Za, Wb[kh]));
    }
    out[k] = p;
    if (kh != k) out[kh] = ph;
    if (S) {
      acc += (k == 0 ? 1.0 : 2.0) * (S[k].x * p.x + S[k].y * p.y);
      if (kh != k) acc += (kh == H ? 1.0 : 2.0) * (S[kh].x * ph.x + S[kh].y * ph.y);
    }
  }
  if (lam_per) {
    const double s = block_sum<1024>(acc, red);
    if (threadIdx.x == 0) lam_per[(size_t)vec * B + m] = s / (double)b;
  }
}

// Time domain -> half spectrum, FP64: sub-transforms of z_r[s] = z[R s + r]
// with z[p] = x[2p] + i x[2p+1]; grid (B, R).
template <int LOGM>
__global__ __launch_bounds__(threads_for_h<double>(LOGM)) void k_sub_gather64(const double* s_time, int b,
                                                                       int Rr, const cx<double>* twM,
                                                                       cx<double>* E) {
  constexpr int M = 1 << LOGM;
  constexpr int NT = threads_for_h<double>(LOGM);
  constexpr int PL = padded_len(M);
  __shared__ __align__(16) double re[2 * PL];
  double* im = re + PL;
  const Soa<double> buf{re, im};
  const int m = blockIdx.x, r = blockIdx.y;
  const double* x = s_time + (size_t)m * b;
  for (int s = threadIdx.x; s < M; s += NT) {
    const size_t p = (size_t)Rr * s + r;
    buf.put(s, cx<double>{x[2 * p], x[2 * p + 1]});
  }
  __syncthreads();
  const Twid<double> tw{twM, nullptr};
  fft_soa<double, LOGM, NT, false>(buf, tw);
  cx<double>* out = E + ((size_t)m * Rr + r) * M;
  for (int k = threadIdx.x; k < M; k += NT) out[k] = buf.get(k);
}

// Half spectrum from the sub-transforms E[m][r][M]: S64 (+)= X, S32 = (float) S64.
// One thread per bin pair (k, H-k), k <= H/2: both recombined values serve
// both outputs.
__global__ void k_combine_r2c(const cx<double>* E, int B, int b, int M, int Rr, const cx<double>* Wb,
                              int accumulate, cx<double>* S64, cx<float>* S32) {
  const int H = b / 2;
  const size_t total = (size_t)B * (H / 2 + 1);
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / (H / 2 + 1)), k = (int)(e % (H / 2 + 1));
    const cx<double>* Em = E + (size_t)m * Rr * M;
    const cx<double> Za = recombine(Em, M, Rr, Wb, b, k), Zb = recombine(Em, M, Rr, Wb, b, (H - k) % H);
    const size_t base = (size_t)m * (H + 1);
    auto put = [&](int kk, cx<double> X) {
      if (accumulate) X = cadd(X, S64[base + kk]);
      S64[base + kk] = X;
      if (S32) S32[base + kk] = cx<float>{(float)X.x, (float)X.y};
    };
    put(k, r2c_post(Za, Zb, Wb[k]));
    if (H - k != k) put(H - k, r2c_post(Zb, Za, Wb[H - k]));
  }
}

// Half spectrum -> time domain, FP64, first stage: A[m][r][k'] (see the top).
__global__ void k_c2r_split_a(const cx<double>* S64, int B, int b, int M, int Rr, const cx<double>* Wb,
                              cx<double>* A) {
  const int H = b / 2;
  const size_t total = (size_t)B * M;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / M), kp = (int)(e % M);
    const cx<double>* S = S64 + (size_t)m * (H + 1);
    for (int r = 0; r < Rr; ++r) {
      cx<double> s = {0.0, 0.0};
      for (int q = 0; q < Rr; ++q) {
        const int k = kp + q * M;
        const cx<double> Y = c2r_pack(S[k], S[H - k], Wb[k]);
        s = cadd(s, cmul(Y, cconj(wfull(Wb, b, (long long)(b / Rr) * r * q))));
      }
      A[((size_t)m * Rr + r) * M + kp] = cmul(s, cconj(wfull(Wb, b, 2LL * r * kp)));
    }
  }
}

// Second stage: z_r = IFFT_M(A_r), x[2p] = 2/b Re z[p], x[2p+1] = 2/b Im z[p], p = R s + r.
template <int LOGM>
__global__ __launch_bounds__(threads_for_h<double>(LOGM)) void k_c2r_split_b(const cx<double>* A, int b,
                                                                      int Rr, const cx<double>* twM,
                                                                      double* s_time) {
  constexpr int M = 1 << LOGM;
  constexpr int NT = threads_for_h<double>(LOGM);
  constexpr int PL = padded_len(M);
  __shared__ __align__(16) double re[2 * PL];
  double* im = re + PL;
  const Soa<double> buf{re, im};
  const int m = blockIdx.x, r = blockIdx.y;
  const cx<double>* src = A + ((size_t)m * Rr + r) * M;
  for (int k = threadIdx.x; k < M; k += NT) buf.put(k, src[k]);
  __syncthreads();
  const Twid<double> tw{twM, nullptr};
  fft_soa<double, LOGM, NT, true>(buf, tw);
  double* x = s_time + (size_t)m * b;
  const double scale = 2.0 / (double)b;
  for (int s = threadIdx.x; s < M; s += NT) {
    const size_t p = (size_t)Rr * s + r;
    const cx<double> z = buf.get(s);
    x[2 * p] = z.x * scale;
    x[2 * p + 1] = z.y * scale;
  }
}

// ---------------------------------------------------------------------------
// FP32 power step at b = 65536 (H = 2M, R = 2) in one launch, one work-group
// per (sketch m, restart tau); the LDS holds one M-point transform at a time:
//   for each count-sketch mode j: E_j,0 = FFT_M(residue 0) in LDS, parked in
//   a global scratch row at the bins k' and M - k' of the quads the thread
//   owns; then E_j,1 = FFT_M(residue 1) in LDS, and per quad of bins
//   {k', H - k', M - k', M + k'} the recombination Z[k] = E_0[k mod M] +-
//   W_H^k E_1[k mod M], the real-input bins X_j and the product
//   P = S conj(X_sa) conj(X_sb) (the first mode's partial product waits in
//   the scratch row);
//   then per quad the c2r packing Y and the inverse split A_r; A_0 goes to
//   LDS (at the positions the thread read, so no other thread is disturbed)
//   and A_1 to the scratch row while z_0 = IFFT_M(A_0) is read off, then
//   z_1 = IFFT_M(A_1) and the read-off of the coordinates whose packed
//   position has residue 1.
// With PRE the work-group first forms u = normalised median of Vprev[tau]
// itself (the median prologue of k_power), so no launch of its own is needed.
// ---------------------------------------------------------------------------
struct SplitOneArgs {
  const uint32_t* hx;
  const uint32_t* hxs;
  const uint32_t* ord;
  int n, B;
  const cx<float>* S;    // [B][H+1]
  const cx<float>* Wb;   // [b]
  const cx<float>* twM;  // pass table of the M-point transform
  const float* Uprev;    // [L][n]
  const float* Uy;       // [L][n] or null (second count sketch's vector; not with PRE)
  const float* Vprev;    // [L][B][n] (PRE)
  float* Ucur;           // [L][n]    (PRE, written by m == 0)
  int32_t* flags;        // [L]       (PRE, nullable)
  float* V;              // [L][B][n]
  double* lam_per;       // [L][B]    (mode 1)
  cx<float>* P;          // [L][B][6][M/2 + 1] scratch, by restart tau (tau0 + blockIdx.y)
  int tau0, mode, u_lds;
  int rd, sa, sb;
};

// LDS of k_power_split1: the reduction words, the M-point buffer and (u_lds) u.
constexpr size_t split1_lds_bytes(int logm, int n, bool u_lds) {
  return 128 + 2 * (size_t)padded_len(1 << logm) * sizeof(float) + (u_lds ? (size_t)n * sizeof(float) : 0);
}

// Threads of k_power_split1 (one work-group per CU: the M-point buffer takes
// most of the LDS).
constexpr int kSplit1Threads = 1024;

template <int LOGM, bool PRE>
__global__ __launch_bounds__(kSplit1Threads) void k_power_split1(SplitOneArgs a) {
  constexpr int M = 1 << LOGM;
  constexpr int H = 2 * M;
  constexpr int NT = kSplit1Threads;
  constexpr int PL = padded_len(M);
  constexpr int QH = M / 2 + 1;        // quads k' = 0 .. M/2
  extern __shared__ __align__(16) unsigned char lds[];
  double* red = reinterpret_cast<double*>(lds);
  float* re = reinterpret_cast<float*>(lds + 128);
  float* im = re + PL;
  float* ul = re + 2 * PL;
  const Soa<float> buf{re, im};
  const int tid = threadIdx.x;
  const int m = blockIdx.x;
  const int tl = blockIdx.y;
  const int tau = a.tau0 + tl;
  const int n = a.n, B = a.B;
  const Twid<float> tw{a.twM, nullptr};
  const cx<float>* S = a.S + (size_t)m * (H + 1);
  const cx<float>* Wb = a.Wb;
  cx<float>* Pq = a.P + ((size_t)tau * B + m) * 6 * (size_t)QH;
  const float* ug = a.Uprev + (size_t)tau * n;

  if constexpr (PRE) {
    const bool ok = median_prologue<float, NT>(a.Vprev, a.Uprev, tau, n, B, ul, re, 2 * PL, red, false);
    if (m == 0) {
      for (int i = tid; i < n; i += NT) a.Ucur[(size_t)tau * n + i] = ul[i];
      if (tid == 0 && !ok && a.flags) a.flags[tau] |= 1;
    }
  } else if (a.u_lds) {
    for (int i = tid; i < n; i += NT) ul[i] = ug[i];
    __syncthreads();
  }
  const bool u_lds = PRE || a.u_lds;

  // The twiddles of quad k' from two table entries, w1 = W_b^k' and
  // w2 = W_b^2k': W_b^(H-k') = -conj(w1), W_b^(M-k') = -i conj(w1),
  // W_b^(M+k') = -i w1 (W_b^H = -1, W_b^M = -i), W_b^(2(M-k')) = -conj(w2)
  // for 0 < k' (W_b^0 = 1 for k' = 0).
  struct QuadTw {
    cx<float> k, Hk, Mk, Mpk, k2, Mk2;
  };
  // Z and X_j of quad {k', H - k', M - k', M + k'} from E_j,0 (ea at k', eb
  // at M - k') and E_j,1 (LDS).
  auto quad_x = [&](int kp, const QuadTw& w, const cx<float> ea, const cx<float> eb, cx<float> (&X)[4]) {
    const int km2 = (M - kp) & (M - 1);
    const cx<float> fa = buf.get(kp), fb = buf.get(km2);
    const cx<float> ta = cmul(w.k2, fa), tb = cmul(w.Mk2, fb);
    const cx<float> a0 = cadd(ea, ta), a1 = csub(ea, ta);  // Z[k'], Z[M + k']
    const cx<float> b0 = cadd(eb, tb), b1 = csub(eb, tb);  // Z[M - k'], Z[H - k'] (k' > 0)
    const cx<float> zk = a0, zMk = kp ? b0 : b1, zHk = kp ? b1 : b0, zMpk = a1;
    X[0] = r2c_post(zk, zHk, w.k);
    X[1] = r2c_post(zHk, zk, w.Hk);
    X[2] = r2c_post(zMk, zMpk, w.Mk);
    X[3] = r2c_post(zMpk, zMk, w.Mpk);
  };
  // Global inputs of one quad: W_b^k', W_b^2k', two values from the scratch
  // row (the parked E_j,0 in slots 4 and 5, or in the second mode the first
  // mode's products in slots 0 to 3 as well), and in the first mode S at the
  // quad's four bins.  The quad loops load quad k' + NT before they store
  // quad k', so that waiting for the loads never waits for the stores.
  struct QuadIn {
    cx<float> w1, w2, ea, eb, v[4];
  };
  auto quad_load = [&](int kp, bool first) -> QuadIn {
    QuadIn in;
    in.w1 = Wb[kp];
    in.w2 = Wb[2 * kp];
    in.ea = Pq[4 * (size_t)QH + kp];
    in.eb = Pq[5 * (size_t)QH + kp];
    if (first) {
      in.v[0] = S[kp];
      in.v[1] = S[H - kp];
      in.v[2] = S[M - kp];
      in.v[3] = S[M + kp];
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) in.v[q] = Pq[(size_t)q * QH + kp];
    }
    return in;
  };
  auto quad_tw_of = [&](int kp, const QuadIn& in) -> QuadTw {
    QuadTw t;
    t.k = in.w1;
    t.Hk = {-in.w1.x, in.w1.y};
    t.Mk = {-in.w1.y, -in.w1.x};
    t.Mpk = {in.w1.y, -in.w1.x};
    t.k2 = in.w2;
    t.Mk2 = kp ? cx<float>{-in.w2.x, in.w2.y} : in.w2;
    return t;
  };
  // First mode: P = S conj(X_sa) into the scratch row.
  auto quad_first = [&](int kp, const QuadIn& in) {
    const QuadTw w = quad_tw_of(kp, in);
    cx<float> X[4];
    quad_x(kp, w, in.ea, in.eb, X);
#pragma unroll
    for (int q = 0; q < 4; ++q) Pq[(size_t)q * QH + kp] = cmulc(in.v[q], X[q]);
  };
  // Second mode: P *= conj(X_sb), the packing Y and the inverse split; A_0
  // into LDS at k' and M - k' (the positions this thread read), A_1 into the
  // scratch row in place of the P values just read (slots 0 and 1).
  auto quad_second = [&](int kp, const QuadIn& in) {
    const QuadTw w = quad_tw_of(kp, in);
    cx<float> X[4];
    quad_x(kp, w, in.ea, in.eb, X);
    cx<float> P[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) P[q] = cmulc(in.v[q], X[q]);
    const cx<float> Ya = c2r_pack(P[0], P[1], w.k);     // Y[k']
    const cx<float> Yc = c2r_pack(P[3], P[2], w.Mpk);   // Y[M + k']
    buf.put(kp, cadd(Ya, Yc));
    Pq[kp] = cmulc(csub(Ya, Yc), w.k2);                 // A_1[k'] = (Ya - Yc) W_H^(-k')
    if (kp > 0 && kp < M / 2) {
      const cx<float> Yb = c2r_pack(P[2], P[3], w.Mk);  // Y[M - k']
      const cx<float> Yd = c2r_pack(P[1], P[0], w.Hk);  // Y[H - k']
      buf.put(M - kp, cadd(Yb, Yd));
      Pq[QH + kp] = cmulc(csub(Yb, Yd), w.Mk2);         // A_1[M - k']
    }
  };
  // The quads of this thread, the next one's loads ahead of this one's stores.
  auto quad_pass = [&](bool first) {
    int kp = tid;
    QuadIn cur = quad_load(kp, first);
    for (; kp <= M / 2; kp += NT) {
      QuadIn nxt = cur;
      if (kp + NT <= M / 2) nxt = quad_load(kp + NT, first);
      if (first) quad_first(kp, cur);
      else quad_second(kp, cur);
      cur = nxt;
    }
  };
  // Count sketch of residue r of mode `mode` (vector uy, else u) and its
  // forward M-point transform in LDS (ends with a barrier).
  auto forward = [&](int mode, const float* uy, int r) {
    zero_lds<NT>(re, 2 * PL * (int)sizeof(float));
    __syncthreads();
    const size_t tb = ((size_t)m * 3 + mode) * n;
    auto getu = [&](uint32_t i) -> float { return uy ? uy[i] : (u_lds ? ul[i] : ug[i]); };
    auto store = [&](uint32_t t, float v) {
      const unsigned p = t >> 1;
      if ((int)(p & 1u) == r) {
        const int q = pidx((int)(p >> 1));
        if (t & 1u) im[q] = v;
        else re[q] = v;
      }
    };
    count_sketch<float>(a.hxs + tb, a.ord + tb, n, NT, getu, store);
    __syncthreads();
    fft_soa<float, LOGM, NT, false>(buf, tw);
  };

  // E_j,0 at the bins k' and M - k' of each quad waits in slots 4 and 5 of
  // the scratch row (each thread reads back what it wrote).
  auto keep_e0 = [&]() {
    for (int kp = tid; kp <= M / 2; kp += NT) {
      Pq[4 * (size_t)QH + kp] = buf.get(kp);
      Pq[5 * (size_t)QH + kp] = buf.get((M - kp) & (M - 1));
    }
    __syncthreads();  // before the next count sketch clears the buffer
  };
  forward(a.sa, nullptr, 0);
  keep_e0();
  forward(a.sa, nullptr, 1);
  quad_pass(true);
  __syncthreads();
  const float* uy = a.Uy ? a.Uy + (size_t)tau * n : nullptr;
  forward(a.sb, uy, 0);
  keep_e0();
  forward(a.sb, uy, 1);
  quad_pass(false);

  // z_r = IFFT_M(A_r) and the read-off of the coordinates of residue r.
  constexpr int RMX = fft_rmax(M, NT);
  constexpr bool PRUNABLE = output_from_groups_ok(M, NT);
  constexpr int NS3 = pass_stride(M, NT, 1);
  const bool prune = PRUNABLE && n * pass_radix(M, NS3, RMX) <= M;
  int om = m, otau = tau;
  asm volatile("" : "+s"(om), "+s"(otau));
  const uint32_t* hx1 = a.hx + ((size_t)om * 3 + a.rd) * n;
  float* Vrow = a.V + ((size_t)otau * B + om) * n;
  const float scale = 2.0f / (float)(2 * H);
  double acc = 0.0;
  auto inverse = [&]() {
    if constexpr (PRUNABLE) {
      fft_soa<float, LOGM, NT, true, false, 2>(buf, tw);
      if (!prune) fft_soa_from<float, LOGM, NT, true, NS3, 0, false>(buf, tw);
    } else {
      fft_soa<float, LOGM, NT, true>(buf, tw);
    }
  };
  auto readoff = [&](int r) {
    for (int i = tid; i < n; i += NT) {
      const uint32_t e = hx1[i];
      const uint32_t t = e >> 1, p = t >> 1;
      if ((int)(p & 1u) != r) continue;
      float val;
      if (PRUNABLE && prune) {
        const cx<float> z = inverse_output_from_groups<float, LOGM, NT>(buf, a.twM, (int)(p >> 1));
        val = (t & 1u) ? z.y : z.x;
      } else {
        const int q = pidx((int)(p >> 1));
        val = (t & 1u) ? im[q] : re[q];
      }
      val *= scale;
      const float v = (e & 1u) ? -val : val;
      Vrow[i] = v;
      acc += (double)(u_lds ? ul[i] : ug[i]) * (double)v;
    }
  };
  constexpr int QP = (M / 2) / NT;  // quads per thread below M/2; k' = M/2 is thread 0's extra
  static_assert((M / 2) % NT == 0, "whole quads per thread");
  __syncthreads();  // A_0 complete in LDS
  inverse();
  // A_1 from the scratch row (written by this thread, program order) into
  // registers; the loads are in flight during the residue-0 read-off.
  cx<float> a1a[QP], a1b[QP], a1m{0.f, 0.f};
#pragma unroll
  for (int q = 0; q < QP; ++q) {
    const int kp = tid + q * NT;
    a1a[q] = Pq[kp];
    a1b[q] = kp > 0 ? Pq[QH + kp] : cx<float>{0.f, 0.f};
  }
  if (tid == 0) a1m = Pq[M / 2];
  readoff(0);
  __syncthreads();  // the residue-0 read-off done
#pragma unroll
  for (int q = 0; q < QP; ++q) {
    const int kp = tid + q * NT;
    buf.put(kp, a1a[q]);
    if (kp > 0) buf.put(M - kp, a1b[q]);
  }
  if (tid == 0) buf.put(M / 2, a1m);
  __syncthreads();
  inverse();
  readoff(1);
  if (a.mode == 1) {
    const double lam = block_sum<NT>(acc, red);
    if (tid == 0) a.lam_per[(size_t)tau * B + m] = lam;
  }
}

}  // namespace tsk
