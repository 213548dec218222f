/*
 * tsk.h -- C ABI of the MI355X (gfx950) sketched tensor CP decomposition library.
 *
 * The library builds tensor sketches of a symmetric 3rd-order tensor and runs
 * the robust tensor power method on them, computing every contraction through
 * FFTs of sketched vectors (Wang, Tung, Smola, Anandkumar, "Fast and
 * Guaranteed Tensor Decomposition via Sketching", NIPS 2015).
 *
 * Conventions shared by every call:
 *   - Pointers are DEVICE pointers unless the argument says "host".  The
 *     caller allocates and owns every buffer passed in; the library owns only
 *     its context, its table objects and internal workspace.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued asynchronously on it.
 *   - Every call validates its arguments on the host before enqueuing any
 *     work and returns a tsk_status; nothing throws across the ABI.  The text
 *     of the last failure on the calling thread is tsk_last_error().
 *   - Indices are 0-based.  The DFT is unnormalised forward,
 *     F(x)_k = sum_t x_t exp(-2 pi i k t / b); the inverse carries 1/b.
 *   - A sketch is stored as its half spectrum, b/2+1 complex values
 *     (interleaved re, im), for each of the B independent sketches:
 *       S64 : double[B][b/2+1][2]  master copy (FP64)
 *       S32 : float [B][b/2+1][2]  working copy used by the FP32 power method
 *   - Limits: 1 <= n <= 65535, b a power of two with 64 <= b <= 65536,
 *     1 <= B <= 64, 1 <= L <= 65535, T >= 1, 1 <= k <= n.  FP64 power
 *     steps and the document build stop at b = 16384.  A power step at
 *     b <= 32768 also needs its work-group's LDS (the half spectrum and the
 *     n-vector) to fit one CU, which bounds n (19348 in FP64 at b = 1024,
 *     23252 in FP32 at b = 16384); requests outside the built kernel
 *     limits return TSK_EUNSUPPORTED.
 */
#ifndef TSK_H
#define TSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSK_OK = 0,
  TSK_EINVAL = -1,       /* null pointer or out-of-range argument          */
  TSK_ESHAPE = -2,       /* sizes inconsistent with the tables / each other */
  TSK_ENOMEM = -3,       /* device workspace allocation failed              */
  TSK_EHIP = -4,         /* a HIP runtime call failed                       */
  TSK_EUNSUPPORTED = -5  /* valid request outside the built kernel limits   */
} tsk_status;

typedef enum { TSK_F32 = 0, TSK_F64 = 1 } tsk_dtype;

typedef struct tsk_ctx* tsk_ctx_t;       /* per-device context + workspace  */
typedef struct tsk_tables* tsk_tables_t; /* device copy of hash/sign tables */
typedef struct tsk_sym_tables* tsk_sym_tables_t; /* colliding-hash tables (Section 3.3) */

/* Library version string (static storage). */
const char* tsk_version(void);

/* Message for the last non-OK status returned on the calling thread. */
const char* tsk_last_error(void);

/* Create a context on HIP device `device`; the device is made current.
 * Destroy frees its workspace.  A context is not thread-safe: calls that
 * share one must be serialised by the caller.  Calls on one context share its
 * internal workspace, so their device work must not overlap either: issue
 * them on one stream, or synchronise between calls on different streams. */
tsk_status tsk_create(tsk_ctx_t* out, int device);
void tsk_destroy(tsk_ctx_t ctx);

/* Launch-shape tuning.  Launch shapes come from fixed rules (mode 0, the
 * default) or from a tuner the library runs on the caller's own data: the
 * dense build's sketches per work-group and slab count (how the buckets are
 * privatised in LDS and how the tensor is split), and the number of restart
 * groups a decomposition runs on parallel graph branches.  Mode 1: the first
 * call of an uncached shape times every candidate twice (blocking on its
 * stream; a decomposition times one-component runs on a copy of the sketch),
 * keeps the rule's shape unless another is faster by more than 3%, and
 * records the choice; mode 2: cached choices
 * only, the rules elsewhere.  cache_path (host, nullable) names a text file,
 * read now and rewritten after each new choice: one line per shape, the key
 * (entry point, device name and CU count, precision, sizes) and the chosen
 * integers.  A choice of build shape changes the rounding of the build within
 * FP64 round-off; restart groups change no result bit.  Errors: TSK_EINVAL
 * (null context, mode). */
tsk_status tsk_tune_config(tsk_ctx_t ctx, int mode, const char* cache_path);

/* Route of the document build (tsk_sketch_build_docs).  Route 1: the
 * per-document transforms of Section 3.2 (three real b-point transforms per
 * document and sketch, six per word).  Route 2: the whitened moment M3(W,W,W)
 * formed as a K^3 FP64 tensor on the matrix cores (about D K^3 / 2
 * multiply-adds over the documents, the same per word), then sketched by
 * Eq. (1) as a dense tensor.  Route 0 (the default) takes the one a cost rule
 * estimates faster: route 2 whenever K^3 is small against B b log2 b.  Both
 * give the same sketch up to rounding.  Route 2 keeps its chunk partial
 * products (at most 256 MB each for the documents and the words) and the K^3
 * tensor in the context's workspace.  Errors: TSK_EINVAL (null context,
 * route outside {0, 1, 2}). */
tsk_status tsk_docs_route(tsk_ctx_t ctx, int route);

/* ---- Randomness (host only, no device work) ------------------------------
 * Hash and sign tables h_j^(m): [n] -> [b], xi_j^(m): [n] -> {+1,-1} for
 * sketch m < B and mode j in {0,1,2} (Algorithm 1, initialisation; the tensor
 * sketch definition of Section 2).  Drawn from SplitMix64 (Steele, Lea and
 * Flood 2014):
 *   r  = mix64(mix64(seed ^ 0x68617368) + (m<<34 | j<<32 | i))
 *   h  = ((r >> 32) * b) >> 32,   xi = bit 31 of r ? -1 : +1
 * where mix64(x) is SplitMix64's output function applied to x.
 * h_host: uint32[B][3][n], xi_host: int8[B][3][n], both host, caller-owned.
 * Errors: TSK_EINVAL for null pointers, n < 1, b < 1, B < 1. */
tsk_status tsk_hash_generate(uint64_t seed, int n, int b, int B,
                             uint32_t* h_host, int8_t* xi_host);

/* Start vectors of the restarts (Algorithm 1, initialisation of each
 * restart: a random point of the unit sphere) for component `comp`:
 *   r_e = mix64(mix64(seed ^ 0x75307530) + (comp<<40 | tau<<20 | 2i+e))
 *   U_e = (r_e >> 11) 2^-53,  z_i = sqrt(-2 ln(1-U_0)) cos(2 pi U_1),
 *   u = z / ||z||.
 * u0_host: double[L][n], host.  Errors: TSK_EINVAL (null, L<1, n<1,
 * L >= 2^20, n >= 2^19). */
tsk_status tsk_init_vectors(uint64_t seed, int comp, int L, int n, double* u0_host);

/* Upload tables (host arrays as produced by tsk_hash_generate, or any table
 * with 0 <= h < b and xi in {+1,-1}) to the context's device and derive the
 * bucket-sorted index order the kernels use for deterministic count
 * sketches.  The tables object owns its device memory until
 * tsk_tables_destroy.  Errors: TSK_EINVAL (range), TSK_EUNSUPPORTED (b). */
tsk_status tsk_tables_create(tsk_ctx_t ctx, int n, int b, int B,
                             const uint32_t* h_host, const int8_t* xi_host,
                             tsk_tables_t* out);
/* Waits for the device, frees the tables and drops the context's recorded
 * decomposition graphs (they hold table addresses).  The context must still
 * be alive. */
void tsk_tables_destroy(tsk_tables_t tab);

/* ---- Sketch construction -------------------------------------------------
 * Dense build, Eq. (1):  s^(m)(t) = sum over (h1(i)+h2(j)+h3(k)) mod b == t of
 * xi1(i) xi2(j) xi3(k) T_ijk, for every m; then S64 = F(s) and S32 = (float)S64.
 * T: [n][n][n] row-major, float (TSK_F32) or double (TSK_F64), n = tables' n.
 * accumulate != 0 adds to S64 instead of overwriting it (the sketch is linear
 * in T, Section 3.1).  Each work-group sums its share of T in 64-bit fixed
 * point (scaled from max |T| so that nothing overflows; repeated builds are
 * bit-identical) and the shares are summed in FP64.  A non-finite entry of T
 * makes every bucket NaN.  The first dense build with a table set also makes
 * its per-fibre offsets (4 B n^2 bytes of device memory, held until
 * tsk_tables_destroy) and waits for its stream once. */
tsk_status tsk_sketch_build_dense(tsk_ctx_t ctx, tsk_tables_t tab, const void* T,
                                  tsk_dtype dtype, double* S64, float* S32,
                                  int accumulate, void* stream);

/* Factor build, Eq. (2) with linearity (Section 3.1):
 *   S64^(m) (+)= sum_r lam_r F(s1 a_r) o F(s2 a_r) o F(s3 a_r),
 * the tensor sum_r lam_r a_r^(x)3 is never formed.  lam: double[k],
 * A: double[k][n] (rows a_r), both device.  All FFTs in FP64. */
tsk_status tsk_sketch_build_factors(tsk_ctx_t ctx, tsk_tables_t tab, const double* lam,
                                    const double* A, int k, double* S64, float* S32,
                                    int accumulate, void* stream);

/* Document build (Appendix D): the B sketches of the whitened third-order
 * moment of spectral LDA, M3(W, W, W), from word counts, never forming a
 * V^3 tensor.  With n the counts of a document of length m >= 3 (shorter
 * documents are dropped), p = W^T n, w_i the i-th row of W, q = W^T M1 (M1
 * the mean of n / m over the kept documents, D of them), a = alpha0/(alpha0+2),
 * c = 2 alpha0^2 / ((alpha0+1)(alpha0+2)):
 *   M3 = (1/D) sum_d [ (p^(x)3 - sum_i n_i (w_i w_i p + w_i p w_i + p w_i w_i)
 *                        + 2 sum_i n_i w_i^(x)3) / (m (m-1)(m-2))
 *                      - a (p p^T - sum_i n_i w_i w_i^T) / (m (m-1)) (x) q  (and its two
 *                        mode permutations) ] + c q^(x)3,
 * the per-document terms by Eq. (td) and the moment combination of
 * Eq. (moment3).  The terms in w_i are gathered per word first (sums over the
 * documents holding it).  Two routes (tsk_docs_route): every rank-1 term
 * sketched by Eq. (2), three transforms per document and sketch and six per
 * word (Section 3.2); or the K^3 tensor formed in FP64 on the matrix cores
 * and sketched by Eq. (1).
 *   rowptr: int32[D+1], col: int32[nnz] word ids in [0, V) (unique within a
 *   document), cnt: int32[nnz] counts >= 1 -- CSR, device.
 *   W: [V][K] in wdtype (TSK_F32 or TSK_F64; the projections p = W^T n, on
 *   the matrix cores, and the transforms run in that precision, the sums over
 *   documents and the moment tensor in FP64), K = the tables' n.
 *   accumulate != 0 adds to S64.  The call reads rowptr[D] back to the host.
 * Errors: TSK_EINVAL (null, D < 1, V < 1, alpha0 < 0 or not finite, dtype),
 * TSK_EUNSUPPORTED (K above 128, or, on the transform route, too large for
 * one work-group's LDS at this b). */
tsk_status tsk_sketch_build_docs(tsk_ctx_t ctx, tsk_tables_t tab, const int32_t* rowptr,
                                 const int32_t* col, const int32_t* cnt, int D, int V,
                                 const void* W, tsk_dtype wdtype, double alpha0, double* S64,
                                 float* S32, int accumulate, void* stream);

/* Spectra from time-domain sketches s_time: double[B][b] (e.g. a sketch kept
 * by the caller), and back.  FP64 throughout. */
tsk_status tsk_sketch_from_time(tsk_ctx_t ctx, int b, int B, const double* s_time,
                                double* S64, float* S32, void* stream);
tsk_status tsk_sketch_export(tsk_ctx_t ctx, int b, int B, const double* S64,
                             double* s_time, void* stream);

/* Deflation (Algorithm 1, deflation step): S64^(m) -= sum_r lam_r
 * F(s1 u_r) o F(s2 u_r) o F(s3 u_r) for the c pairs (lam_r, u_r), then
 * S32 = (float)S64.  lam: double[c], U: double[c][n], device.  FP64. */
tsk_status tsk_sketch_deflate(tsk_ctx_t ctx, tsk_tables_t tab, const double* lam,
                              const double* U, int c, double* S64, float* S32,
                              void* stream);

/* ---- Contractions ---------------------------------------------------------
 * One power step for L vectors (Algorithm 1 inner loop, Proposition 1):
 *   sbar = F^-1( S^(m) o conj F(s2 u) o conj F(s3 u) ),  v^(m)_i = xi1(i) sbar[h1(i)]
 *   vbar_i = med_m v^(m)_i,  u_out = vbar / ||vbar||.
 * Even B takes the mean of the two middle values.  If ||vbar|| is zero or not
 * finite, u_out = u_in and flags[tau] gets bit 0 set (flags are OR-ed, not
 * cleared).  dtype TSK_F32 reads S32 and float vectors; TSK_F64 reads S64
 * and double vectors.  U_in, U_out: [L][n] (may not alias).  V: nullable
 * [L][B][n] per-sketch estimates.  flags: nullable int32[L]. */
tsk_status tsk_power_update(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                            const double* S64, const float* S32, int L,
                            const void* U_in, void* U_out, void* V, int32_t* flags,
                            void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): the power step of
 * tsk_power_update, same kernels and bit-identical results, without the
 * per-sketch estimates argument.  It allocates nothing: the estimates (and, at
 * b = 65536 in FP32, the split step's scratch rows) live in a static 32 MiB
 * device array of the library, one per GPU, held until the process ends; the
 * twiddle tables were made by tsk_tables_create.  Needs
 * L*B*n*sizeof(dtype) bytes (rounded up to 256), plus at b = 65536 in FP32
 * L*B*393264 bytes; more than 32 MiB is TSK_EINVAL.  Every call on one GPU shares
 * that array and leaves its contents behind, so calls that overlap on one GPU
 * (other streams, other threads, other contexts) race: serialise them.  Other
 * arguments and errors as tsk_power_update; a path that would allocate
 * returns TSK_EUNSUPPORTED instead. */
tsk_status tsk_power_update_noalloc(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                    const double* S64, const float* S32, int L,
                                    const void* U_in, void* U_out, int32_t* flags,
                                    void* stream);

/* The median and normalisation of a power step on given per-sketch estimates
 * (Algorithm 1): vbar_i = med_m V[tau][m][i] (odd B: rank (B-1)/2; even B: the
 * mean of ranks B/2-1 and B/2; any NaN among the B values gives NaN), then
 * U_out[tau] = vbar / ||vbar||, or U_in[tau] with flags[tau] |= 1 when
 * ||vbar|| is zero or not finite.  V: [L][B][n], U_in, U_out: [L][n], all
 * device, float for TSK_F32 and double for TSK_F64 (U_out may not alias V or
 * U_in); flags: nullable int32[L], device.  1 <= B <= 64 by sorting networks,
 * larger B by ranking.  Errors: TSK_EINVAL (null, L, n or B < 1, alias,
 * dtype). */
tsk_status tsk_median_normalize(tsk_ctx_t ctx, tsk_dtype dtype, int L, int n, int B,
                                const void* V, const void* U_in, void* U_out,
                                int32_t* flags, void* stream);

/* Per-sketch estimates of T(I,u,u) for L vectors (Proposition 1), without
 * the median: V[tau][m][i] = xi1(i) sbar[h1(i)],
 * sbar = F^-1( S^(m) o conj F(s2 u) o conj F(s3 u) ).  One kernel launch
 * over all L x B (restart, sketch) pairs.  U: [L][n], V: [L][B][n] in dtype. */
tsk_status tsk_contract_tiuu(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                             const double* S64, const float* S32, int L, const void* U,
                             void* V, void* stream);

/* T(u,u,u) estimates for L vectors (Eq. (3) with X = u(x)u(x)u):
 *   lam_per[tau][m] = <s^(m), s^(m)(u^(x)3)> = sum_i u_i v^(m)_i(u),
 *   lam_med[tau] = med_m lam_per[tau][m].
 * U: [L][n] in dtype.  lam_med: double[L]; lam_per: nullable double[L][B]. */
tsk_status tsk_contract_uuu(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                            const double* S64, const float* S32, int L, const void* U,
                            double* lam_med, double* lam_per, void* stream);

/* ---- Fast ALS (Appendix C, Algorithm 2) -----------------------------------
 * Two-vector contraction (Proposition 1 with the two count sketches of
 * different vectors): per sketch m, with a = (rd+1) mod 3, c = (rd+2) mod 3,
 *   sbar = F^-1( S^(m) o conj F(s_a X[r]) o conj F(s_c Y[r]) ),
 *   V[r][m][i] = xi_rd(i) sbar[h_rd(i)],
 * the estimate of T contracted with X[r] in mode a and Y[r] in mode c, read
 * off in mode rd (rd = 0: T(I, x, y)).  X, Y: [L][n], V: [L][B][n], device,
 * float for TSK_F32 (reads S32, any b) and double for TSK_F64 (reads S64,
 * b <= 16384).  Errors: TSK_EINVAL (null, rd, L), TSK_EUNSUPPORTED (b). */
tsk_status tsk_contract_two(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                            const double* S64, const float* S32, int rd, int L,
                            const void* X, const void* Y, void* V, void* stream);

/* Algorithm 2 for a rank-k CP model (factors held as rows: F[f][r] is column
 * r of A, B, C for f = 0, 1, 2): T sweeps, each updating A, B, C in turn by
 *   A = G^+ Vbar,  Vbar[r] = med_m V[r][m] (tsk_contract_two, rd = 0),
 *   G = (B B^T) o (C C^T)  (k x k, pseudo-inverse over eigenvalues
 *   > 1e-12 of the largest), lambda_r = ||A[r]||, A[r] /= lambda_r,
 * and B, C likewise with the modes rotated (the update equation of
 * Appendix C; the printed Algorithm 2 omits the pseudo-inverse, which is the
 * identity for orthonormal factors).  Power-kernel precision as dtype; the
 * factors, G and the update in FP64.  F0: double[3][k][n] initial factors;
 * F_out: double[3][k][n] (may equal F0); lam_out: double[k] from the last (C)
 * update; all device.  1 <= k <= 64, T >= 1, b as tsk_contract_two.
 * Errors: TSK_EINVAL, TSK_EUNSUPPORTED (b). */
tsk_status tsk_als(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, const double* S64,
                   const float* S32, int k, int T, const double* F0, double* lam_out,
                   double* F_out, void* stream);

/* ---- Colliding-hash symmetric sketches (Section 3.3, Eq. (5); Appendix B) --
 * One hash h: [n] -> [b] and one sign sigma(i) = i^q(i), q in {0,1,2,3}, per
 * sketch (h_host [B][n] in [0,b), q_host [B][n], host).  The sketch of a
 * symmetric tensor
 *   s(t) = sum over (h(i)+h(j)+h(k)) mod b == t of sigma(i) sigma(j) sigma(k) T_ijk
 * is complex; it is kept in the time domain (s64 FP64, s32 FP32 copy,
 * [B][b][2]) and as its full spectrum (S64, S32, [B][b][2]), all device,
 * caller-owned.  b a power of two in [256, 65536] (from 32768 on the power
 * step runs through split transforms and a device buffer of
 * 6 L B 16384 (b = 32768) or 12 L B 16384 (b = 65536) bytes of workspace).
 * Errors: TSK_EINVAL, TSK_EUNSUPPORTED (b). */
tsk_status tsk_sym_tables_create(tsk_ctx_t ctx, int n, int b, int B, const uint32_t* h_host,
                                 const uint8_t* q_host, tsk_sym_tables_t* out);
void tsk_sym_tables_destroy(tsk_sym_tables_t tab);

/* Dense build of Eq. (5) from the entries T[i][j][k] with i <= j <= k, each
 * weighted by the number of distinct orderings of (i, j, k) (6, 3 or 1; for a
 * symmetric tensor, as Section 3.3 assumes, this is the sum over all entries,
 * and only those entries are read), accumulated in
 * 64-bit fixed point (a power-of-two scale from max |T|; repeated builds are
 * bit-identical), then S64 = F(s64), S32 = (float)S64, s32 = (float)s64
 * (s32, S32 nullable).  T: [n][n][n] row-major, float or double by dtype.
 * accumulate != 0 adds to s64.  A non-finite entry makes the sketch NaN.
 * The first build with a table set also makes its per-pair codes (2 B n^2
 * bytes of device memory, held until tsk_sym_tables_destroy) and waits for
 * its stream once. */
tsk_status tsk_sym_sketch_build_dense(tsk_ctx_t ctx, tsk_sym_tables_t tab, const void* T,
                                      tsk_dtype dtype, double* s64, float* s32, double* S64,
                                      float* S32, int accumulate, void* stream);

/* Per-sketch estimates V[tau][m][i] = Re v_i of T(I,u,u) for L vectors
 * (Appendix B read-off with weight 1/3 on all four terms; FP32):
 *   v_i = (1/3) [ conj(s_i) (c1 + c2)[h_i] / 2 + conj(s_i^2) u_i c3[2h_i]
 *                 + conj(s_i^3) u_i^2 s[3h_i] ],  s_i = sigma(i),
 *   c1 + c2 = F^-1(S o (conj(U1)^2 + conj(U2))), c3 = F^-1(S o conj(U1)),
 *   U1 = F(sum_{h(i)=t} s_i u_i), U2 = F(sum_{2h(i)=t} s_i^2 u_i^2).
 * S32, s32: [B][b][2]; U: float [L][n]; V: float [L][B][n]; device.
 * n at most about 2800 at b >= 16384 (LDS).  Errors: TSK_EINVAL,
 * TSK_EUNSUPPORTED. */
tsk_status tsk_sym_contract_tiuu(tsk_ctx_t ctx, tsk_sym_tables_t tab, const float* S32,
                                 const float* s32, int L, const float* U, float* V, void* stream);

/* Algorithm 1 on symmetric sketches: per component, T power steps (FP32
 * read-offs, median over sketches of Re v, normalisation; zero or
 * non-finite medians keep the vector and set flags[c][tau]), selection by the
 * median of u . Re v (lowest restart on ties), lambda_hat = med_m Re <s, s_X>
 * in FP64 at the FP64-renormalised winner (s_X the sketch of the upper
 * triangle of u^(x)3, Appendix B), and deflation of s64/s32/S64/S32 by
 * lambda_hat (s_u * s_u * s_u).  u0: nullable double [k][L][n] (null: the
 * start vectors of tsk_init_vectors(seed)); lam_out double[k]; U_out double
 * [k][n]; tau_out, flags_out nullable int32 [k], [k][L]; device. */
tsk_status tsk_sym_decompose(tsk_ctx_t ctx, tsk_sym_tables_t tab, double* s64, float* s32,
                             double* S64, float* S32, int k, int L, int T, const double* u0,
                             uint64_t seed, double* lam_out, double* U_out, int32_t* tau_out,
                             int32_t* flags_out, void* stream);

/* ---- Fast spectral LDA (Appendix D, Algorithm 3) ---------------------------
 * Whitening from the empirical second moment (Eq. (moment2)):
 *   M2 = (1/D) sum_d (n_d n_d^T - diag n_d)/(m_d (m_d - 1)) - alpha0/(alpha0+1) M1 M1^T
 * over the documents with at least three words (M1 the mean of n_d/m_d),
 * never formed: a randomized truncated SVD by subspace iteration,
 *   Y = M2 Omega; `iters` times { Q = orth(Y); Y = M2 Q }; Q = orth(Y);
 *   B = Q^T M2 Q = E diag(d) E^T;  W = Q E diag(1/sqrt|d|), sigma = |d|,
 * columns by decreasing |d| (orth: Q = Y E_G diag(1/sqrt(d_G)) from the
 * eigenpairs of Y^T Y).  Then W^T M2 W = I on the captured subspace.
 * CSR counts as tsk_sketch_build_docs; Omega: double [V][K] start block
 * (drawn by the caller, e.g. Gaussian); W_out double [V][K]; sigma_out
 * double [K]; device.  1 <= K <= 100, K <= V.  Errors: TSK_EINVAL. */
tsk_status tsk_lda_whiten(tsk_ctx_t ctx, const int32_t* rowptr, const int32_t* col,
                          const int32_t* cnt, int D, int V, int K, double alpha0,
                          const double* Omega, int iters, double* W_out, double* sigma_out,
                          void* stream);

/* Algorithm 3's output from the CP decomposition (lam [k], U [k][K] rows
 * v_i) of M3(W, W, W):
 *   alpha_i = 4 alpha0 (alpha0 + 1) / ((alpha0 + 2)^2 lam_i^2),
 *   mu_i = (alpha0 + 2)/2 lam_i (W^+)^T v_i,  (W^+)^T = W (W^T W)^+,
 * the pseudo-inverse over eigenvalues above 1e-12 of the largest.  W double
 * [V][K]; lam double [k]; U double [k][K]; alpha_out double [k]; mu_out
 * double [k][V]; device.  1 <= K <= 100.  Errors: TSK_EINVAL. */
tsk_status tsk_lda_recover(tsk_ctx_t ctx, int V, int K, int k, double alpha0, const double* W,
                           const double* lam, const double* U, double* alpha_out, double* mu_out,
                           void* stream);

/* Held-out likelihood of a topic model (Section 5.2).  For each document d
 * of a CSR corpus (counts n, length m) the mixing vector
 *   pi_d = argmin { ||n/m - Phi pi||_2 : pi >= 0, sum_k pi_k = 1 }
 * (simplex-constrained least squares, solved exactly by the primal
 * active-set method on G = Phi^T Phi, one work-group per document) and its
 * average log-likelihood L_d = (1/m) sum_i n_i ln(sum_k pi_k Phi[w_i][k]).
 *   rowptr int32[D+1], col int32[nnz], cnt int32[nnz] (CSR, device);
 *   Phi double [V][K] topics as columns (full column rank; entries positive
 *   where documents have words, else L_d = -inf); pi_out double [D][K];
 *   ll_out double [D]; device.  L_d is NaN for a document without words or
 *   one the method did not finish in 10 K + 10 steps.  1 <= K <= min(V, 128).
 *   The call reads rowptr[D] back to the host.
 * Errors: TSK_EINVAL (null, sizes). */
tsk_status tsk_lda_heldout(tsk_ctx_t ctx, const int32_t* rowptr, const int32_t* col,
                           const int32_t* cnt, int D, int V, int K, const double* Phi,
                           double* pi_out, double* ll_out, void* stream);

/* ---- Gradients (extensions built on Eq. (3) and Proposition 1) ----------
 * f(u) = med_m f^(m)(u) with f^(m)(u) = <s^(m), s_1(u) * s_2(u) * s_3(u)>, the
 * T(u,u,u) estimate of Eq. (3), and its gradient.  Each count sketch is linear
 * in u, so
 *   d f^(m) / d u_i = sum_j xi_j(i) corr(s^(m), s_a(u) * s_b(u))[h_j(i)]
 * ({a, b} the two other modes): every term is the read-off of Proposition 1
 * with mode j in the place of mode 1.  The median's gradient is that of the
 * sketch it selects (even B: the mean of the two middle sketches; ranks break
 * ties by sketch index).
 *   U: [L][n] in dtype.  scale: nullable [L] in dtype, multiplies grad[tau].
 *   f_med: double[L].  f_per: nullable double[L][B].  grad: [L][n] in dtype.
 * Errors as tsk_power_update. */
tsk_status tsk_contract_tuuu_grad(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                  const double* S64, const float* S32, int L, const void* U,
                                  const void* scale, double* f_med, double* f_per, void* grad,
                                  void* stream);

/* Sketched CP loss: the least-squares objective of the CP decomposition
 * (Section 2) measured through the B sketches, using their linearity
 * (Section 3.1):
 *   r^(m) = s^(m)(T) - sum_i lam_i s^(m)(u_i (x) u_i (x) u_i)
 *   loss  = (1/B) sum_m ||r^(m)||^2
 *   d loss / d lam_i = -(2/B) sum_m <r^(m), s^(m)(u_i (x) u_i (x) u_i)>
 *   d loss / d u_i   = -(2/B) lam_i sum_m sum_j xi_j corr(r^(m), s_a(u_i) * s_b(u_i))[h_j]
 * S64: sketches of T (read only).  lam: [k], U: [k][n] in dtype.  scale:
 * nullable device scalar in dtype multiplying both gradients.  loss: double[1].
 * grad_lam: nullable [k], grad_U: nullable [k][n], in dtype; with both NULL
 * only the loss is computed.  The residual spectra are formed in FP64 (FP32
 * inputs are widened first); the gradient read-offs run in dtype.
 * Errors: TSK_EINVAL (null S64/lam/U/loss, k outside [1, 65535], dtype). */
tsk_status tsk_cp_loss(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, const double* S64, int k,
                       const void* lam, const void* U, const void* scale, double* loss,
                       void* grad_lam, void* grad_U, void* stream);

/* ---- Decomposition --------------------------------------------------------
 * Algorithm 1 for k components: per component, L restarts x T power steps on
 * the sketches (all restarts and sketches batched in each launch), selection
 * tau* = argmax_tau med_m T(u_T,u_T,u_T)^(m) (lowest tau on ties; non-finite
 * values never win), u_hat = u_T^(tau*) renormalised in FP64,
 * lam_hat = med_m <s^(m), s^(m)(u_hat^(x)3)> in FP64, deflation of S64 in FP64
 * and refresh of S32.  The launches are recorded once per shape into a HIP
 * graph and replayed.
 *   dtype: precision of the power steps (TSK_F32 uses S32, TSK_F64 uses S64).
 *   S64/S32: in: sketches of the tensor; out: sketches of the deflated tensor.
 *   u0: nullable double[k][L][n]; NULL draws them with tsk_init_vectors(seed, c, ...).
 *   lam_out: double[k]; U_out: double[k][n]; tau_out: nullable int32[k];
 *   flags_out: nullable int32[k][L] (bit 0: a zero/non-finite median vector).
 * plain != 0 runs the comparison path: one launch per (restart, step) with B
 * work-groups each, no batching across restarts and no graph. */
tsk_status tsk_decompose(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                         double* S64, float* S32, int k, int L, int T,
                         const double* u0, uint64_t seed, double* lam_out,
                         double* U_out, int32_t* tau_out, int32_t* flags_out,
                         int plain, void* stream);

/* One instance of a batched decomposition: the arguments of tsk_decompose
 * (pointers inside are device pointers, owned by the caller; plain = 0). */
typedef struct {
  tsk_tables_t tab;     /* the instance's tables (created on the same context) */
  tsk_dtype dtype;      /* precision of its power steps */
  double* S64;          /* its sketches, deflated in place */
  float* S32;
  int k, L, T;
  const double* u0;     /* nullable double[k][L][n] */
  uint64_t seed;        /* start vectors when u0 is NULL */
  double* lam_out;      /* double[k] */
  double* U_out;        /* double[k][n] */
  int32_t* tau_out;     /* nullable int32[k] */
  int32_t* flags_out;   /* nullable int32[k][L] */
} tsk_problem;

/* Algorithm 1 for `ninst` independent instances of different sizes (n, k, b,
 * B, dtype may all differ), each exactly as tsk_decompose computes it.  The
 * instances are spread, longest first, over up to 32 branches of one HIP
 * graph (recorded once per set of shapes and buffers and replayed), so the
 * device runs several instances' launches at once.  probs: host array of
 * `ninst` problems; the library keeps one workspace for all of them.
 * Errors: TSK_EINVAL (ninst < 1, null, or an instance failing the checks of
 * tsk_decompose; the message names the instance). */
tsk_status tsk_decompose_batched(tsk_ctx_t ctx, int ninst, const tsk_problem* probs, void* stream);

/* Device workspace, in bytes, that tsk_decompose_batched keeps for `probs`. */
tsk_status tsk_workspace_size(tsk_ctx_t ctx, int ninst, const tsk_problem* probs, size_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* TSK_H */
