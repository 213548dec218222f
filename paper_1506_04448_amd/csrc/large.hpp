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
// FP32 power step at b = 65536 (H = 2M, R = 2) in three launches:
//   k_sub_cs        E_j,r = FFT_M of the count sketches of u (modes sa, sb)
//   k_power_split_mid  per quad of bins {k', M-k', M+k', H-k'}: Z, X_j, the
//                   product P = S conj(X_sa) conj(X_sb), its c2r packing Y
//                   and the inverse split A_r
//   k_power_split_out  z_r = IFFT_M(A_r) and the read-off of the coordinates
//                   whose packed position has residue r.
// ---------------------------------------------------------------------------
struct SplitMidArgs {
  const cx<float>* E;   // [nvec][B][2][2][M]
  const cx<float>* S;   // [B][H+1]
  const cx<float>* Wb;  // [b]
  int B, b, M;
  cx<float>* A;         // [nvec][B][2][M]
};

__global__ __launch_bounds__(256) void k_power_split_mid(SplitMidArgs a) {
  const int m = blockIdx.x, vec = blockIdx.y;
  const int M = a.M, H = 2 * M;
  const cx<float>* E2 = a.E + (((size_t)vec * a.B + m) * 2 + 0) * 2 * (size_t)M;
  const cx<float>* E3 = a.E + (((size_t)vec * a.B + m) * 2 + 1) * 2 * (size_t)M;
  const cx<float>* S = a.S + (size_t)m * (H + 1);
  cx<float>* A0 = a.A + (((size_t)vec * a.B + m) * 2 + 0) * (size_t)M;
  cx<float>* A1 = A0 + M;
  // Z[km] and Z[km + M] from the two sub-transforms (W_H^km E_1[km] added or
  // subtracted), km < M.
  auto zpair = [&](const cx<float>* E, int km, cx<float>& lo, cx<float>& hi) {
    const cx<float> t = cmul(a.Wb[2 * km], E[M + km]);
    lo = cadd(E[km], t);
    hi = csub(E[km], t);
  };
  auto Y = [&](int k, cx<float> Pk, cx<float> PHk) -> cx<float> { return c2r_pack(Pk, PHk, a.Wb[k]); };
  for (int kp = blockIdx.z * blockDim.x + threadIdx.x; kp <= M / 2; kp += gridDim.z * blockDim.x) {
    // The quad k', H - k', M - k', M + k' needs Z at those four bins, which
    // come from the sub-transform bins k' and M - k' (mod M).
    const int km2 = (M - kp) % M;
    cx<float> P[4];  // at k', H - k', M - k', M + k'
    const cx<float>* Es[2] = {E2, E3};
    cx<float> X[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cx<float> a0, a1, b0, b1;
      zpair(Es[j], kp, a0, a1);    // Z[k'], Z[M + k']
      zpair(Es[j], km2, b0, b1);   // Z[M - k'], Z[H - k'] (k' > 0); Z[0], Z[M] (k' = 0)
      const cx<float> zk = a0, zMk = kp ? b0 : b1, zHk = kp ? b1 : b0, zMpk = a1;
      X[j][0] = r2c_post(zk, zHk, a.Wb[kp]);
      X[j][1] = r2c_post(zHk, zk, a.Wb[H - kp]);
      X[j][2] = r2c_post(zMk, zMpk, a.Wb[M - kp]);
      X[j][3] = r2c_post(zMpk, zMk, a.Wb[M + kp]);
    }
    const int ks[4] = {kp, H - kp, M - kp, M + kp};
#pragma unroll
    for (int q = 0; q < 4; ++q) P[q] = cmulc(cmulc(S[ks[q]], X[0][q]), X[1][q]);
    const cx<float> Pa = P[0], Pd = P[1], Pb = P[2], Pc = P[3];
    const cx<float> Ya = Y(kp, Pa, Pd);              // Y[k']
    const cx<float> Yc = Y(M + kp, Pc, Pb);          // Y[M + k']
    A0[kp] = cadd(Ya, Yc);
    A1[kp] = cmulc(csub(Ya, Yc), a.Wb[2 * kp]);      // * W_H^(-k')
    if (kp > 0 && kp < M / 2) {
      const cx<float> Yb = Y(M - kp, Pb, Pc);        // Y[M - k']
      const cx<float> Yd = Y(H - kp, Pd, Pa);        // Y[H - k']
      A0[M - kp] = cadd(Yb, Yd);
      A1[M - kp] = cmulc(csub(Yb, Yd), a.Wb[2 * (M - kp)]);
    }
  }
}

struct SplitOutArgs {
  const cx<float>* A;     // [nvec][B][2][M]
  const uint32_t* hx;
  int n, B, rd, M, b;
  const cx<float>* twM;
  float* V;               // [nvec][B][n]
};

template <int LOGM>
__global__ __launch_bounds__(threads_for_h<float>(LOGM)) void k_power_split_out(SplitOutArgs a) {
  constexpr int M = 1 << LOGM;
  constexpr int NT = threads_for_h<float>(LOGM);
  constexpr int PL = padded_len(M);
  __shared__ __align__(16) float re[2 * PL];
  float* im = re + PL;
  const Soa<float> buf{re, im};
  const int m = blockIdx.x, vec = blockIdx.y, r = blockIdx.z;
  const cx<float>* src = a.A + (((size_t)vec * a.B + m) * 2 + r) * (size_t)M;
  for (int k = threadIdx.x; k < M; k += NT) buf.put(k, src[k]);
  __syncthreads();
  const Twid<float> tw{a.twM, nullptr};
  const int n = a.n;
  // With n small against M the transform leaves out its last two passes and
  // the read-off forms each output it needs from the groups before them.
  constexpr int RMX = fft_rmax(M, NT);
  constexpr bool PRUNABLE = output_from_groups_ok(M, NT);
  constexpr int NS3 = pass_stride(M, NT, 1);
  const bool prune = PRUNABLE && n * pass_radix(M, NS3, RMX) <= M;
  if constexpr (PRUNABLE) {
    fft_soa<float, LOGM, NT, true, true, 2>(buf, tw);
    if (!prune) fft_soa_from<float, LOGM, NT, true, NS3, 0, true>(buf, tw);
  } else {
    fft_soa<float, LOGM, NT, true>(buf, tw);
  }
  const uint32_t* hx1 = a.hx + ((size_t)m * 3 + a.rd) * n;
  float* Vrow = a.V + ((size_t)vec * a.B + m) * n;
  const float scale = 2.0f / (float)a.b;
  for (int i = threadIdx.x; i < n; i += NT) {
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
    Vrow[i] = (e & 1u) ? -val : val;
  }
}

// lam_per[vec][m] = sum_i u_vec[i] V[vec][m][i] (FP64 sum); one block per (m, vec).
template <typename R>
__global__ __launch_bounds__(256) void k_rowdot(const R* U, const R* V, int n, int B, double* lam_per) {
  __shared__ double red[4];
  const int m = blockIdx.x, vec = blockIdx.y;
  const R* u = U + (size_t)vec * n;
  const R* v = V + ((size_t)vec * B + m) * n;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += (double)u[i] * (double)v[i];
  const double s = block_sum<256>(acc, red);
  if (threadIdx.x == 0) lam_per[(size_t)vec * B + m] = s;
}

}  // namespace tsk
