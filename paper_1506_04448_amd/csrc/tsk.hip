// Host side of the C ABI: context, tables, validation, kernel launches and
// the decompose loop (recorded into a HIP graph once per shape).
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstring>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <map>
#include <mutex>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/tsk.h"
#include "kernels.hpp"
#include "large.hpp"
#include "symmetric.hpp"
#include "spectral.hpp"
#include "moment.hpp"

#include <rocprim/device/device_radix_sort.hpp>
#include "status.hpp"

using tsk::cx;

// Device memory of the allocation-free power step (tsk_power_update_noalloc):
// per-sketch estimates and, at b = 65536, the split transforms' buffers.  Each
// GPU the library runs on holds its own copy until the process ends; host
// code reaches it only through the address hipGetSymbolAddress returns.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace tsk {
char* last_error_buffer() {
  static thread_local char buf[512] = {0};
  return buf;
}
}  // namespace tsk

#define TSK_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return tsk::fail(TSK_EHIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                             \
  } while (0)

#define TSK_TRY(expr)              \
  do {                             \
    tsk_status s_ = (expr);        \
    if (s_ != TSK_OK) return s_;   \
  } while (0)

namespace {

constexpr int kMinLogB = 6;
constexpr int kMaxLogB = 16;
// Up to this size every FP64 transform fits one work-group's LDS; longer ones
// are split by residue into sub-transforms of 2^kSubLogM64 points (large.hpp).
constexpr int kLdsLogB = 14;
constexpr int kSubLogM64 = 13;
constexpr int kSubLogM64Mid = 11;  // forward FP64 transforms at b = 16384
constexpr int kSubLogM32 = 14;     // FP32 power steps at b = 65536

int ilog2_exact(int b) {
  if (b <= 0 || (b & (b - 1))) return -1;
  int l = 0;
  while ((1 << l) < b) ++l;
  return l;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct GraphEntry {
  std::vector<uint64_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct tsk_ctx {
  int device = 0;
  hipStream_t cap = nullptr;
  std::map<int, void*> tw64, tw32;
  std::map<int, void*> wb64, wb32;   // full-circle tables W_b^x, x < b
  std::map<int, DevBuf> ws;          // named workspaces
  std::vector<GraphEntry> graphs;
  std::vector<uint64_t> u0_key;      // cached generated start vectors
  std::vector<uint64_t> u0b_key;     // the same for batched decompositions
  std::vector<hipStream_t> fork;     // branch streams of batched graphs
  std::vector<hipEvent_t> fork_ev;   // one event per branch, plus the fork event
  std::vector<hipStream_t> gfork;    // restart-group branches of one decomposition
  std::vector<hipEvent_t> gfork_ev;
  void* scratch = nullptr;           // this device's address of `scratch` below
  bool no_alloc = false;             // set while an allocation-free entry point runs
  // Launch-shape tuning (tsk_tune_config): mode, cache file, the choices by
  // shape key, the device's name in every key, and a restart-group count
  // forced while a decomposition's candidates are timed.
  int tune_mode = 0;
  std::string tune_path;
  std::map<std::string, std::vector<int>> tune;
  std::string tune_dev;
  int force_groups = 0;
  int docs_route = 0;  // tsk_docs_route: 0 rule, 1 transforms, 2 moment tensor
};

struct tsk_tables {
  tsk_ctx* ctx = nullptr;
  int n = 0, b = 0, B = 0, logb = 0;
  uint32_t* hx = nullptr;
  uint32_t* hxs = nullptr;
  uint32_t* ord = nullptr;
  // Bin offsets of the first two modes per (i, j) fibre and sketch, made by
  // the first dense build ([B][efs] words).
  uint32_t* ef = nullptr;
  long long efs = 0;
};

// Colliding-hash tables: one (h, q) per index and sketch, plus the entries
// sorted by p h mod b (stable by index) for p = 1, 2, 3.
struct tsk_sym_tables {
  tsk_ctx* ctx = nullptr;
  int n = 0, b = 0, B = 0, logb = 0;
  uint32_t* hq = nullptr;    // [B][n] (h << 2) | q
  uint32_t* srt = nullptr;   // [3][B][n] (p h mod b << 2) | p q mod 4
  uint32_t* ord = nullptr;   // [3][B][n]
  uint32_t* ef = nullptr;    // [B][pairs + pad] pair codes, made by the first build
};

namespace {

enum WsId {
  WS_PARTIAL = 0, WS_STIME, WS_PROD, WS_U, WS_V, WS_LAMPER, WS_LAMMED, WS_CNT, WS_FLAGS,
  WS_UHAT, WS_LAM64, WS_U0, WS_LAMHAT, WS_AMAX, WS_V3, WS_R64, WS_R32, WS_LAMD, WS_UD, WS_BATCH,
  WS_DOCS, WS_SPLIT, WS_SPLITP, WS_ALS, WS_SYM, WS_LDA, WS_LDAR, WS_TUNE, WS_HELD, WS_SYMSPLIT, WS_GRAM
};

void clear_graphs(tsk_ctx* c) {
  for (auto& g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  c->graphs.clear();
}

// Grow-only device workspace.  Growing drains the device first and drops
// recorded graphs, which may point at the old buffer.  Counter workspaces are
// zero-filled on allocation; kernels return them to zero after use.
tsk_status ws_get(tsk_ctx* c, int id, size_t bytes, void** out) {
  DevBuf& d = c->ws[id];
  if (bytes == 0) bytes = 256;
  if (d.bytes < bytes) {
    if (c->no_alloc)
      return tsk::fail(TSK_EUNSUPPORTED, "allocation-free call would allocate a %zu-byte workspace", bytes);
    TSK_HIP(hipDeviceSynchronize());
    clear_graphs(c);
    if (d.p) TSK_HIP(hipFree(d.p));
    d.p = nullptr;
    d.bytes = 0;
    size_t nb = std::max(bytes, (size_t)4096);
    if (hipMalloc(&d.p, nb) != hipSuccess) {
      d.p = nullptr;
      return tsk::fail(TSK_ENOMEM, "workspace allocation of %zu bytes failed", nb);
    }
    TSK_HIP(hipMemset(d.p, 0, nb));
    TSK_HIP(hipDeviceSynchronize());
    d.bytes = nb;
    // A new buffer may reuse a freed address: start vectors cached under an
    // address are uploaded again.
    c->u0_key.clear();
    c->u0b_key.clear();
  }
  *out = d.p;
  return TSK_OK;
}

// exp(-2 pi i j / M) in FP64, exact on the axes.
static void unit_root(long j, long M, double* cs, double* sn) {
  j %= M;
  if (j < 0) j += M;
  if (j == 0) { *cs = 1.0; *sn = 0.0; }
  else if (4 * j == M) { *cs = 0.0; *sn = -1.0; }
  else if (2 * j == M) { *cs = -1.0; *sn = 0.0; }
  else if (4 * j == 3 * M) { *cs = 0.0; *sn = 1.0; }
  else {
    const double a = 6.283185307179586476925286766559 * (double)j / (double)M;
    *cs = cos(a);
    *sn = -sin(a);
  }
}

// Twiddle table of a length-b real transform (see fft.hpp, Twid): the per-pass
// table of the H = b/2 point complex FFT as run by `nt` threads (the radix
// plan depends on it; 0 = the power kernel's thread count), then W_b^k for
// k = 0..H.  Computed in FP64, rounded once to R; one table per (b, nt).
template <typename R>
tsk_status get_tw(tsk_ctx* c, int logb, const cx<R>** out, int nt = 0) {
  auto& mp = (sizeof(R) == 8) ? c->tw64 : c->tw32;
  if (nt == 0) nt = tsk::power_threads<R>(logb - 1);
  const int key = (logb << 16) | nt;
  auto it = mp.find(key);
  if (it == mp.end()) {
    if (c->no_alloc)
      return tsk::fail(TSK_EUNSUPPORTED, "allocation-free call would allocate the b=2^%d twiddle table", logb);
    const int b = 1 << logb, H = b / 2;
    const int NT = nt;
    const int rmax = tsk::fft_rmax(H, NT);
    const int plen = tsk::pass_table_len(H, NT);
    std::vector<cx<R>> h(tsk::twid_len(H, NT));
    int off = 0;
    for (int ns = 1; ns < H;) {
      const int rad = tsk::pass_radix(H, ns, rmax);
      if (ns > 1) {
        for (int r = 1; r < rad; ++r)
          for (int k = 0; k < ns; ++k) {
            double cs, sn;
            unit_root((long)r * k, (long)ns * rad, &cs, &sn);
            h[off + (r - 1) * ns + k] = cx<R>{(R)cs, (R)sn};
          }
        off += (rad - 1) * ns;
      }
      ns *= rad;
    }
    if (off != plen) return tsk::fail(TSK_EHIP, "internal: twiddle plan mismatch");
    for (int k = 0; k <= H; ++k) {
      double cs, sn;
      unit_root(k, b, &cs, &sn);
      h[plen + k] = cx<R>{(R)cs, (R)sn};
    }
    void* d = nullptr;
    TSK_HIP(hipMalloc(&d, sizeof(cx<R>) * h.size()));
    TSK_HIP(hipMemcpy(d, h.data(), sizeof(cx<R>) * h.size(), hipMemcpyHostToDevice));
    it = mp.emplace(key, d).first;
  }
  *out = reinterpret_cast<const cx<R>*>(it->second);
  return TSK_OK;
}

// W_b^x for x in [0, b), computed in FP64 and rounded once to R.
template <typename R>
tsk_status get_wb(tsk_ctx* c, int logb, const cx<R>** out) {
  auto& mp = (sizeof(R) == 8) ? c->wb64 : c->wb32;
  auto it = mp.find(logb);
  if (it == mp.end()) {
    if (c->no_alloc)
      return tsk::fail(TSK_EUNSUPPORTED, "allocation-free call would allocate the b=2^%d root table", logb);
    const int b = 1 << logb;
    std::vector<cx<R>> h(b);
    for (int x = 0; x < b; ++x) {
      double cs, sn;
      unit_root(x, b, &cs, &sn);
      h[x] = cx<R>{(R)cs, (R)sn};
    }
    void* d = nullptr;
    TSK_HIP(hipMalloc(&d, sizeof(cx<R>) * h.size()));
    TSK_HIP(hipMemcpy(d, h.data(), sizeof(cx<R>) * h.size(), hipMemcpyHostToDevice));
    it = mp.emplace(logb, d).first;
  }
  *out = reinterpret_cast<const cx<R>*>(it->second);
  return TSK_OK;
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

tsk_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return tsk::fail(TSK_EHIP, "%s launch failed: %s", what, hipGetErrorString(e));
  return TSK_OK;
}

// ---- launch helpers dispatching on log2 b -----------------------------------

// LDS of one CU on gfx950, the most one work-group can use.
constexpr size_t kMaxLds = 160 * 1024;

template <typename R, int LOGB, bool PRE>
tsk_status launch_power_v(const tsk::PowerArgs<R>& a, size_t lds, int B, int nrest, hipStream_t st) {
  constexpr int NT = tsk::power_threads<R>(LOGB - 1);
  // Allow the full LDS as dynamic shared memory, once per device and kernel.
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_power<R, LOGB, PRE>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL((tsk::k_power<R, LOGB, PRE>), dim3(B, nrest), dim3(NT), lds, st, a);
  return check_launch("k_power");
}

// LDS plan of a power step: table rows in LDS when two work-groups still fit
// a CU with them (or one fits only with them), else without; n too large
// for the vector alone is unsupported.
template <typename R>
tsk_status power_lds_plan(int logb, int n, size_t* bytes, int* tab) {
  const size_t with = tsk::power_lds_bytes<R>(logb - 1, n, true);
  const size_t without = tsk::power_lds_bytes<R>(logb - 1, n, false);
  if (with <= kMaxLds / 2 || (without > kMaxLds / 2 && with <= kMaxLds)) {
    *bytes = with;
    *tab = 1;
  } else if (without <= kMaxLds) {
    *bytes = without;
    *tab = 0;
  } else {
    return tsk::fail(TSK_EUNSUPPORTED,
                     "power step: n=%d needs %zu bytes of LDS at b=2^%d in this precision (max %zu)", n,
                     without, logb, kMaxLds);
  }
  return TSK_OK;
}

template <typename R>
tsk_status median_norm_launch(const R* V, const R* Uin, R* Uout, int32_t* flags, int L, int n, int B,
                              hipStream_t st) {
  hipLaunchKernelGGL((tsk::k_median_norm<R>), dim3(L), dim3(tsk::median_threads<R>()), 0, st, V, Uin, Uout, flags, n,
                     B);
  return check_launch("k_median_norm");
}

// The median of the previous step runs as the power kernel's prologue when it
// is cheap there (B <= 16 values per coordinate, at most two coordinates per
// thread, all of them staged in the sequence buffer at once): every one of the
// B work-groups of a restart repeats it.  Otherwise it is a launch of its own,
// once per restart, before a power launch that reads the medians.
template <typename R, int LOGB>
bool fused_median(int n, int B) {
  constexpr int NT = tsk::power_threads<R>(LOGB - 1);
  const long staged = 2L * tsk::padded_len(1 << (LOGB - 1));
  return B <= 16 && n <= 2 * NT && (long)n * (B + 2) <= staged;
}

template <typename R, int LOGB>
tsk_status launch_power_t(tsk::PowerArgs<R> a, int B, int nrest, hipStream_t st) {
  size_t lds = 0;
  TSK_TRY(power_lds_plan<R>(LOGB, a.n, &lds, &a.tab_lds));
  if (a.prefix && !fused_median<R, LOGB>(a.n, B)) {
    const size_t on = (size_t)a.tau0 * a.n, obn = on * B;
    TSK_TRY(median_norm_launch<R>(a.Vprev + obn, a.Uprev + on, a.Ucur + on,
                                  a.flags ? a.flags + a.tau0 : nullptr, nrest, a.n, B, st));
    a.prefix = 0;
    a.Uprev = a.Ucur;
  }
  if (a.prefix) return launch_power_v<R, LOGB, true>(a, lds, B, nrest, st);
  return launch_power_v<R, LOGB, false>(a, lds, B, nrest, st);
}

template <typename R>
tsk_status launch_power(int logb, const tsk::PowerArgs<R>& a, int B, int nrest, hipStream_t st) {
  switch (logb) {
    case 6: return launch_power_t<R, 6>(a, B, nrest, st);
    case 7: return launch_power_t<R, 7>(a, B, nrest, st);
    case 8: return launch_power_t<R, 8>(a, B, nrest, st);
    case 9: return launch_power_t<R, 9>(a, B, nrest, st);
    case 10: return launch_power_t<R, 10>(a, B, nrest, st);
    case 11: return launch_power_t<R, 11>(a, B, nrest, st);
    case 12: return launch_power_t<R, 12>(a, B, nrest, st);
    case 13: return launch_power_t<R, 13>(a, B, nrest, st);
    case 14: return launch_power_t<R, 14>(a, B, nrest, st);
    case 15:
      if constexpr (sizeof(R) == 4) return launch_power_t<R, 15>(a, B, nrest, st);
      break;
    default: break;
  }
  return tsk::fail(TSK_EUNSUPPORTED, "power step: b=2^%d not built in this precision", logb);
}

template <int LOGB>
tsk_status launch_rank1_t(const tsk::Rank1Args& a, int B, int c, hipStream_t st) {
  constexpr int NT = tsk::threads_for_h<double>(LOGB - 1);
  hipLaunchKernelGGL((tsk::k_rank1<LOGB>), dim3(B, c), dim3(NT), 0, st, a);
  return check_launch("k_rank1");
}
template <int LOGB>
tsk_status launch_r2c_t(const double* s, cx<double>* S64, cx<float>* S32, const cx<double>* tw,
                        int acc, int B, hipStream_t st) {
  constexpr int NT = tsk::threads_for_h<double>(LOGB - 1);
  hipLaunchKernelGGL((tsk::k_r2c64<LOGB>), dim3(B), dim3(NT), 0, st, s, S64, S32, tw, acc);
  return check_launch("k_r2c64");
}
template <int LOGB>
tsk_status launch_c2r_t(const cx<double>* S64, double* s, const cx<double>* tw, int B,
                        hipStream_t st) {
  constexpr int NT = tsk::threads_for_h<double>(LOGB - 1);
  hipLaunchKernelGGL((tsk::k_c2r64<LOGB>), dim3(B), dim3(NT), 0, st, S64, s, tw);
  return check_launch("k_c2r64");
}

#define TSK_LOGB_SWITCH(logb, CALL)                   \
  switch (logb) {                                     \
    case 6: return CALL(6);                           \
    case 7: return CALL(7);                           \
    case 8: return CALL(8);                           \
    case 9: return CALL(9);                           \
    case 10: return CALL(10);                         \
    case 11: return CALL(11);                         \
    case 12: return CALL(12);                         \
    case 13: return CALL(13);                         \
    case 14: return CALL(14);                         \
    default: break;                                   \
  }

// b <= 8192 (longer ones go through the sub-transform kernels).
tsk_status launch_rank1(int logb, const tsk::Rank1Args& a, int B, int c, hipStream_t st) {
  switch (logb) {
    case 6: return launch_rank1_t<6>(a, B, c, st);
    case 7: return launch_rank1_t<7>(a, B, c, st);
    case 8: return launch_rank1_t<8>(a, B, c, st);
    case 9: return launch_rank1_t<9>(a, B, c, st);
    case 10: return launch_rank1_t<10>(a, B, c, st);
    case 11: return launch_rank1_t<11>(a, B, c, st);
    case 12: return launch_rank1_t<12>(a, B, c, st);
    case 13: return launch_rank1_t<13>(a, B, c, st);
    default: break;
  }
  return tsk::fail(TSK_EUNSUPPORTED, "rank-1 spectra: b=2^%d not built", logb);
}
tsk_status launch_r2c(int logb, const double* s, cx<double>* S64, cx<float>* S32,
                      const cx<double>* tw, int acc, int B, hipStream_t st) {
#define CALL(L) launch_r2c_t<L>(s, S64, S32, tw, acc, B, st)
  TSK_LOGB_SWITCH(logb, CALL)
#undef CALL
  return tsk::fail(TSK_EUNSUPPORTED, "r2c: b=2^%d not built", logb);
}
tsk_status launch_c2r(int logb, const cx<double>* S64, double* s, const cx<double>* tw, int B,
                      hipStream_t st) {
#define CALL(L) launch_c2r_t<L>(S64, s, tw, B, st)
  TSK_LOGB_SWITCH(logb, CALL)
#undef CALL
  return tsk::fail(TSK_EUNSUPPORTED, "c2r: b=2^%d not built", logb);
}

int grid_for(size_t count, int threads) {
  size_t g = (count + threads - 1) / threads;
  return (int)std::min<size_t>(std::max<size_t>(g, 1), 65536);
}

// ---- transforms longer than one work-group's LDS (see large.hpp) ------------

int sub_R64(int logb) { return 1 << (logb - 1 - kSubLogM64); }

// Rank-1 spectra through the sub-transform kernels: from b = 16384 on, where
// one mode's transform per work-group (three per sketch) beats one
// work-group doing all three in sequence.
bool rank1_split_path(int logb) { return logb >= kLdsLogB; }

// Sub-transform buffer of the split rank-1 spectra of c vectors.
size_t rank1_split_bytes(tsk_tables_t tab, int c) {
  return (size_t)c * tab->B * 3 * sub_R64(tab->logb) * ((size_t)1 << kSubLogM64) * sizeof(cx<double>);
}

// Tables the split paths read, uploaded outside any graph capture.
tsk_status preload_split_tables(tsk_ctx_t ctx, int logb, bool fp32_power) {
  if (!rank1_split_path(logb)) return TSK_OK;
  const cx<double>* t64 = nullptr;
  const cx<double>* w64 = nullptr;
  TSK_TRY(get_tw<double>(ctx, kSubLogM64 + 1, &t64, tsk::threads_for_h<double>(kSubLogM64)));
  TSK_TRY(get_wb<double>(ctx, logb, &w64));
  if (fp32_power) {
    const cx<float>* t32 = nullptr;
    const cx<float>* w32 = nullptr;
    TSK_TRY(get_tw<float>(ctx, kSubLogM32 + 1, &t32, tsk::kSplit1Threads));
    TSK_TRY(get_wb<float>(ctx, logb, &w32));
  }
  return TSK_OK;
}

// prod / lam_per of Rank1Args a for c vectors through the split transforms.
tsk_status rank1_split(tsk_ctx_t ctx, tsk_tables_t tab, const tsk::Rank1Args& a, int c, void* Ebuf,
                       hipStream_t st) {
  if (!Ebuf) return tsk::fail(TSK_EHIP, "internal: split rank-1 buffer missing");
  const int Rr = sub_R64(tab->logb), M = 1 << kSubLogM64;
  const cx<double>* twM = nullptr;
  const cx<double>* Wb = nullptr;
  TSK_TRY(get_tw<double>(ctx, kSubLogM64 + 1, &twM, tsk::threads_for_h<double>(kSubLogM64)));
  TSK_TRY(get_wb<double>(ctx, tab->logb, &Wb));
  tsk::SubCsArgs<double, double> sa;
  sa.hxs = tab->hxs;
  sa.ord = tab->ord;
  sa.n = tab->n;
  sa.B = tab->B;
  sa.Rr = Rr;
  sa.nmodes = 3;
  sa.mode[0] = 0;
  sa.mode[1] = 1;
  sa.mode[2] = 2;
  sa.U = a.U;
  sa.U2 = nullptr;
  sa.twM = twM;
  sa.E = reinterpret_cast<cx<double>*>(Ebuf);
  hipLaunchKernelGGL((tsk::k_sub_cs<double, kSubLogM64, double>), dim3(tab->B, c, 3 * Rr),
                     dim3(tsk::threads_for_h<double>(kSubLogM64)), 0, st, sa);
  TSK_TRY(check_launch("k_sub_cs"));
  hipLaunchKernelGGL(tsk::k_combine_rank1, dim3(tab->B, c), dim3(1024), 0, st,
                     (const cx<double>*)Ebuf, tab->B, tab->b, M, Rr, Wb, a.S64, a.prod, a.lam_per);
  return check_launch("k_combine_rank1");
}

tsk_status launch_rank1_any(tsk_ctx_t ctx, tsk_tables_t tab, const tsk::Rank1Args& a, int c, void* Ebuf,
                            hipStream_t st) {
  if (!rank1_split_path(tab->logb)) return launch_rank1(tab->logb, a, tab->B, c, st);
  return rank1_split(ctx, tab, a, c, Ebuf, st);
}

// Time domain -> half spectrum (FP64) at any supported b.
tsk_status r2c_any(tsk_ctx_t ctx, int logb, const double* s, cx<double>* S64, cx<float>* S32, int acc,
                   int B, hipStream_t st) {
  if (logb < kLdsLogB) {
    const cx<double>* tw = nullptr;
    TSK_TRY(get_tw<double>(ctx, logb, &tw));
    return launch_r2c(logb, s, S64, S32, tw, acc, B, st);
  }
  // At b = 16384 the transform still fits one work-group, but B work-groups
  // leave the chip idle: four sub-transforms per sketch finish sooner.
  const int logm = logb > kLdsLogB ? kSubLogM64 : kSubLogM64Mid;
  const int Rr = 1 << (logb - 1 - logm), M = 1 << logm, b = 1 << logb;
  const int nt = tsk::threads_for_h<double>(logm);
  const cx<double>* twM = nullptr;
  const cx<double>* Wb = nullptr;
  TSK_TRY(get_tw<double>(ctx, logm + 1, &twM, nt));
  TSK_TRY(get_wb<double>(ctx, logb, &Wb));
  void* E = nullptr;
  TSK_TRY(ws_get(ctx, WS_SPLITP, (size_t)B * Rr * M * sizeof(cx<double>), &E));
  if (logm == kSubLogM64)
    hipLaunchKernelGGL((tsk::k_sub_gather64<kSubLogM64>), dim3(B, Rr), dim3(nt), 0, st, s, b, Rr, twM,
                       (cx<double>*)E);
  else
    hipLaunchKernelGGL((tsk::k_sub_gather64<kSubLogM64Mid>), dim3(B, Rr), dim3(nt), 0, st, s, b, Rr, twM,
                       (cx<double>*)E);
  TSK_TRY(check_launch("k_sub_gather64"));
  hipLaunchKernelGGL(tsk::k_combine_r2c, dim3(grid_for((size_t)B * (b / 2 + 1), 256)), dim3(256), 0, st,
                     (const cx<double>*)E, B, b, M, Rr, Wb, acc, S64, S32);
  return check_launch("k_combine_r2c");
}

// Half spectrum -> time domain (FP64) at any supported b.
tsk_status c2r_any(tsk_ctx_t ctx, int logb, const cx<double>* S64, double* s, int B, hipStream_t st) {
  if (logb <= kLdsLogB) {
    const cx<double>* tw = nullptr;
    TSK_TRY(get_tw<double>(ctx, logb, &tw));
    return launch_c2r(logb, S64, s, tw, B, st);
  }
  const int Rr = sub_R64(logb), M = 1 << kSubLogM64, b = 1 << logb;
  const cx<double>* twM = nullptr;
  const cx<double>* Wb = nullptr;
  TSK_TRY(get_tw<double>(ctx, kSubLogM64 + 1, &twM, tsk::threads_for_h<double>(kSubLogM64)));
  TSK_TRY(get_wb<double>(ctx, logb, &Wb));
  void* A = nullptr;
  TSK_TRY(ws_get(ctx, WS_SPLITP, (size_t)B * Rr * M * sizeof(cx<double>), &A));
  hipLaunchKernelGGL(tsk::k_c2r_split_a, dim3(grid_for((size_t)B * M, 256)), dim3(256), 0, st, S64, B, b, M,
                     Rr, Wb, (cx<double>*)A);
  TSK_TRY(check_launch("k_c2r_split_a"));
  hipLaunchKernelGGL((tsk::k_c2r_split_b<kSubLogM64>), dim3(B, Rr),
                     dim3(tsk::threads_for_h<double>(kSubLogM64)), 0, st, (const cx<double>*)A, b, Rr,
                     twM, s);
  return check_launch("k_c2r_split_b");
}

// Buffer of the FP32 split power step (b = 65536) for nvec vectors: per
// (vector, sketch) 6 (M/2 + 1) values (the first mode's partial spectral
// product, the residue-0 sub-transform between its two uses, A_1).
struct SplitBufs {
  void* A = nullptr;  // cx<float>[nvec][B][6][M/2 + 1]
};
size_t power_split_bytes_A(tsk_tables_t tab, int nvec) {
  return (size_t)nvec * tab->B * 6 * (((size_t)1 << kSubLogM32) / 2 + 1) * sizeof(cx<float>);
}
bool needs_power_split(tsk_tables_t tab, tsk_dtype dtype) {
  return dtype == TSK_F32 && tab->logb > kLdsLogB + 1;
}

tsk_status check_tables(tsk_tables_t tab, tsk_ctx_t ctx, const char* fn) {
  if (!ctx) return tsk::fail(TSK_EINVAL, "%s: null context", fn);
  if (!tab) return tsk::fail(TSK_EINVAL, "%s: null tables", fn);
  if (tab->ctx != ctx) return tsk::fail(TSK_EINVAL, "%s: tables belong to another context", fn);
  return TSK_OK;
}

tsk_status set_device(tsk_ctx_t ctx) {
  TSK_HIP(hipSetDevice(ctx->device));
  return TSK_OK;
}

// Device address of `scratch` on `device`, which must be current: looked up
// once per device and kept.
constexpr int kScratchDevices = 64;
tsk_status scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[kScratchDevices] = {};
  if (device < 0 || device >= kScratchDevices)
    return tsk::fail(TSK_EUNSUPPORTED, "device %d: scratch kept for devices below %d", device, kScratchDevices);
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return tsk::fail(TSK_EHIP, "scratch address on device %d: %s", device, hipGetErrorString(e));
    addr[device] = p;
  }
  *out = addr[device];
  return TSK_OK;
}

// Twiddle tables of the power step at this b, so that later steps (and the
// allocation-free one) find them made.
tsk_status preload_power_tables(tsk_ctx_t ctx, int logb) {
  if (logb <= kLdsLogB + 1) {
    const cx<float>* t32 = nullptr;
    TSK_TRY(get_tw<float>(ctx, logb, &t32));
  }
  if (logb <= kLdsLogB) {
    const cx<double>* t64 = nullptr;
    TSK_TRY(get_tw<double>(ctx, logb, &t64));
  }
  return preload_split_tables(ctx, logb, logb > kLdsLogB + 1);
}

// Marks a context as forbidden to allocate for the lifetime of the guard.
struct NoAllocGuard {
  tsk_ctx* c;
  explicit NoAllocGuard(tsk_ctx* ctx) : c(ctx) { c->no_alloc = true; }
  ~NoAllocGuard() { c->no_alloc = false; }
};

// ---- launch-shape tuning ------------------------------------------------------
// Shapes the tuner chooses: sketches per work-group and slab count of the
// dense build (how the buckets are privatised in LDS and how the tensor is
// split), and the number of restart groups a decomposition runs on parallel
// graph branches.  A choice is stored under a key naming the device, the
// entry point, the precision and the sizes that decide it; the cache file has
// one line per key: the key, then the chosen integers.

std::string tune_key(tsk_ctx_t ctx, const char* what, tsk_dtype dtype, std::initializer_list<long> sizes) {
  std::ostringstream k;
  k << what << ':' << ctx->tune_dev << ':' << (dtype == TSK_F32 ? "f32" : "f64");
  for (long v : sizes) k << ':' << v;
  return k.str();
}

void tune_load(tsk_ctx_t ctx) {
  std::ifstream f(ctx->tune_path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream ls(line);
    std::string key;
    if (!(ls >> key)) continue;
    std::vector<int> v;
    int x;
    while (ls >> x) v.push_back(x);
    if (!v.empty()) ctx->tune[key] = v;
  }
}

tsk_status tune_save(tsk_ctx_t ctx) {
  if (ctx->tune_path.empty()) return TSK_OK;
  const std::string tmp = ctx->tune_path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return tsk::fail(TSK_EINVAL, "tuning cache %s: cannot write", tmp.c_str());
    for (const auto& kv : ctx->tune) {
      f << kv.first;
      for (int x : kv.second) f << ' ' << x;
      f << '\n';
    }
    if (!f) return tsk::fail(TSK_EINVAL, "tuning cache %s: write failed", tmp.c_str());
  }
  if (std::rename(tmp.c_str(), ctx->tune_path.c_str()) != 0)
    return tsk::fail(TSK_EINVAL, "tuning cache %s: rename failed", ctx->tune_path.c_str());
  return TSK_OK;
}

// Mean time in ms of `reps` runs of `run` on stream st, after one untimed run.
template <typename F>
tsk_status time_runs(hipStream_t st, int reps, F run, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  TSK_HIP(hipEventCreate(&e0));
  TSK_HIP(hipEventCreate(&e1));
  tsk_status s = run();
  if (s == TSK_OK && hipEventRecord(e0, st) != hipSuccess) s = tsk::fail(TSK_EHIP, "tuning: event record");
  for (int r = 0; r < reps && s == TSK_OK; ++r) s = run();
  if (s == TSK_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                      hipEventElapsedTime(ms, e0, e1) != hipSuccess))
    s = tsk::fail(TSK_EHIP, "tuning: event timing");
  if (s == TSK_OK) *ms /= (float)reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

// The cached choice of `key`, or, in mode 1 and when not cached, the fastest
// candidate (timed by time_one) recorded under it; nullptr means "use the rule".
template <typename C, typename F>
tsk_status tune_choose(tsk_ctx_t ctx, const std::string& key, const std::vector<C>& cands,
                       std::vector<int> (*encode)(const C&), F time_one, const std::vector<int>** out) {
  *out = nullptr;
  if (ctx->tune_mode == 0) return TSK_OK;
  auto it = ctx->tune.find(key);
  if (it == ctx->tune.end() && ctx->tune_mode == 1 && !cands.empty()) {
    // Two passes over the candidates, each keeping its faster time (drift
    // between candidates averages out); cands[0] is the rule, and another
    // candidate replaces it only when faster by more than 3% (timing noise
    // of a few per cent must not move the choice off the rule).
    std::vector<float> t(cands.size(), 0.0f);
    for (int pass = 0; pass < 2; ++pass)
      for (size_t i = 0; i < cands.size(); ++i) {
        float ms = 0.0f;
        TSK_TRY(time_one(cands[i], &ms));
        t[i] = pass == 0 ? ms : std::min(t[i], ms);
      }
    size_t bi = 0;
    for (size_t i = 1; i < cands.size(); ++i)
      if (t[i] < 0.97f * t[0] && t[i] < t[bi]) bi = i;
    it = ctx->tune.emplace(key, encode(cands[bi])).first;
    TSK_TRY(tune_save(ctx));
  }
  if (it != ctx->tune.end()) *out = &it->second;
  return TSK_OK;
}

}  // namespace

// =============================================================================
// Context and tables
// =============================================================================

extern "C" const char* tsk_version(void) { return "tsk 0.1 (gfx950)"; }
extern "C" const char* tsk_last_error(void) { return tsk::last_error_buffer(); }

extern "C" tsk_status tsk_create(tsk_ctx_t* out, int device) {
  if (!out) return tsk::fail(TSK_EINVAL, "tsk_create: null output");
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1)
    return tsk::fail(TSK_EHIP, "tsk_create: no HIP device available");
  if (device < 0 || device >= count)
    return tsk::fail(TSK_EINVAL, "tsk_create: device %d out of range [0,%d)", device, count);
  TSK_HIP(hipSetDevice(device));
  void* scr = nullptr;
  TSK_TRY(scratch_address(device, &scr));
  tsk_ctx* c = new tsk_ctx();
  c->device = device;
  c->scratch = scr;
  if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return tsk::fail(TSK_EHIP, "tsk_create: stream creation failed");
  }
  *out = c;
  return TSK_OK;
}

extern "C" void tsk_destroy(tsk_ctx_t c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  clear_graphs(c);
  for (auto& kv : c->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& kv : c->tw64) (void)hipFree(kv.second);
  for (auto& kv : c->tw32) (void)hipFree(kv.second);
  for (auto& kv : c->wb64) (void)hipFree(kv.second);
  for (auto& kv : c->wb32) (void)hipFree(kv.second);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  for (auto s : c->fork) (void)hipStreamDestroy(s);
  for (auto e : c->fork_ev) (void)hipEventDestroy(e);
  for (auto s : c->gfork) (void)hipStreamDestroy(s);
  for (auto e : c->gfork_ev) (void)hipEventDestroy(e);
  delete c;
}

extern "C" tsk_status tsk_tune_config(tsk_ctx_t ctx, int mode, const char* cache_path) {
  if (!ctx) return tsk::fail(TSK_EINVAL, "tsk_tune_config: null context");
  if (mode < 0 || mode > 2) return tsk::fail(TSK_EINVAL, "tsk_tune_config: mode %d not in {0, 1, 2}", mode);
  TSK_TRY(set_device(ctx));
  hipDeviceProp_t prop;
  TSK_HIP(hipGetDeviceProperties(&prop, ctx->device));
  std::string arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == ' ') ch = '_';
  ctx->tune_dev = arch + "_cu" + std::to_string(prop.multiProcessorCount);
  ctx->tune_mode = mode;
  ctx->tune_path = cache_path ? cache_path : "";
  ctx->tune.clear();
  if (!ctx->tune_path.empty()) tune_load(ctx);
  return TSK_OK;
}

extern "C" tsk_status tsk_docs_route(tsk_ctx_t ctx, int route) {
  if (!ctx) return tsk::fail(TSK_EINVAL, "tsk_docs_route: null context");
  if (route < 0 || route > 2) return tsk::fail(TSK_EINVAL, "tsk_docs_route: route %d not in {0, 1, 2}", route);
  ctx->docs_route = route;
  return TSK_OK;
}

extern "C" tsk_status tsk_tables_create(tsk_ctx_t ctx, int n, int b, int B, const uint32_t* h_host,
                                        const int8_t* xi_host, tsk_tables_t* out) {
  if (!out) return tsk::fail(TSK_EINVAL, "tsk_tables_create: null output");
  *out = nullptr;
  if (!ctx || !h_host || !xi_host) return tsk::fail(TSK_EINVAL, "tsk_tables_create: null argument");
  if (n < 1 || n > 65535) return tsk::fail(TSK_EINVAL, "tsk_tables_create: n=%d outside [1,65535]", n);
  if (B < 1 || B > 64) return tsk::fail(TSK_EINVAL, "tsk_tables_create: B=%d outside [1,64]", B);
  const int logb = ilog2_exact(b);
  if (logb < 0) return tsk::fail(TSK_EINVAL, "tsk_tables_create: b=%d is not a power of two", b);
  if (logb < kMinLogB || logb > kMaxLogB)
    return tsk::fail(TSK_EUNSUPPORTED, "tsk_tables_create: b=%d outside [64,65536]", b);
  const size_t cnt = (size_t)B * 3 * n;
  std::vector<uint32_t> hx(cnt), hxs(cnt), ord(cnt);
  for (size_t e = 0; e < cnt; ++e) {
    if (h_host[e] >= (uint32_t)b)
      return tsk::fail(TSK_EINVAL, "tsk_tables_create: h[%zu]=%u >= b=%d", e, h_host[e], b);
    if (xi_host[e] != 1 && xi_host[e] != -1)
      return tsk::fail(TSK_EINVAL, "tsk_tables_create: xi[%zu]=%d not +-1", e, (int)xi_host[e]);
    hx[e] = (h_host[e] << 1) | (xi_host[e] < 0 ? 1u : 0u);
  }
  std::vector<uint32_t> idx(n);
  for (int mj = 0; mj < 3 * B; ++mj) {
    const size_t base = (size_t)mj * n;
    std::iota(idx.begin(), idx.end(), 0u);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t p, uint32_t q) {
      return (hx[base + p] >> 1) < (hx[base + q] >> 1);
    });
    for (int p = 0; p < n; ++p) {
      ord[base + p] = idx[p];
      hxs[base + p] = hx[base + idx[p]];
    }
  }
  TSK_TRY(set_device(ctx));
  tsk_tables* t = new tsk_tables();
  t->ctx = ctx;
  t->n = n;
  t->b = b;
  t->B = B;
  t->logb = logb;
  void* p = nullptr;
  if (hipMalloc(&p, 3 * cnt * sizeof(uint32_t)) != hipSuccess) {
    delete t;
    return tsk::fail(TSK_ENOMEM, "tsk_tables_create: device allocation failed");
  }
  t->hx = reinterpret_cast<uint32_t*>(p);
  t->hxs = t->hx + cnt;
  t->ord = t->hxs + cnt;
  hipError_t e1 = hipMemcpy(t->hx, hx.data(), cnt * 4, hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(t->hxs, hxs.data(), cnt * 4, hipMemcpyHostToDevice);
  hipError_t e3 = hipMemcpy(t->ord, ord.data(), cnt * 4, hipMemcpyHostToDevice);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    (void)hipFree(p);
    delete t;
    return tsk::fail(TSK_EHIP, "tsk_tables_create: upload failed");
  }
  const tsk_status ps = preload_power_tables(ctx, logb);
  if (ps != TSK_OK) {
    (void)hipFree(p);
    delete t;
    return ps;
  }
  *out = t;
  return TSK_OK;
}

extern "C" void tsk_tables_destroy(tsk_tables_t t) {
  if (!t) return;
  (void)hipSetDevice(t->ctx->device);
  (void)hipDeviceSynchronize();
  // Recorded graphs hold this table's device addresses; a later table could
  // reuse the handle's address and match their keys.
  clear_graphs(t->ctx);
  (void)hipFree(t->hx);
  if (t->ef) (void)hipFree(t->ef);
  delete t;
}

// =============================================================================
// Sketch construction
// =============================================================================

namespace {

// Two static-LDS pool sizes of the dense build (64-bit words): the whole CU
// (one work-group per CU) and 20 KB (several per CU) for small sketches.
constexpr int kBuildPoolLarge = (159 * 1024) / 8;  // leaves room for the reduction scratch
constexpr int kBuildPoolSmall = (20 * 1024) / 8;

template <typename TIn, bool SYM>
tsk_status launch_build(bool small, bool split, int nblk, const tsk::BuildArgs<TIn>& a, hipStream_t st) {
  if (small)
    hipLaunchKernelGGL((tsk::k_build_dense<TIn, kBuildPoolSmall, false, SYM>), dim3(nblk), dim3(1024), 0, st, a);
  else if (split)
    hipLaunchKernelGGL((tsk::k_build_dense<TIn, kBuildPoolLarge, true, SYM>), dim3(nblk), dim3(1024), 0, st, a);
  else
    hipLaunchKernelGGL((tsk::k_build_dense<TIn, kBuildPoolLarge, false, SYM>), dim3(nblk), dim3(1024), 0, st, a);
  return check_launch("k_build_dense");
}

// Slabs of the dense build: a multiple of 8 (one per XCD lane of the grid
// mapping), never slabs of fewer than 8 fibres; the fewest whose
// work-groups (ngroups per slab) fill 90% of the rounds they take (one
// work-group per CU with the large pool, two with the small one), else the
// count that fills them best.
int pick_nslab(long long nfib, int ngroups, bool small) {
  const long long per_round = 256LL * (small ? 2 : 1);
  int best = 8;
  double best_fill = -1.0;
  for (int ns = 8; ns <= 1024 && (ns == 8 || nfib / ns >= 8); ns += 8) {
    const long long w = (long long)ns * ngroups;
    const double fill = (double)w / (double)(per_round * ((w + per_round - 1) / per_round));
    if (fill > best_fill + 1e-9) {
      best_fill = fill;
      best = ns;
    }
    if (fill >= 0.9) break;
  }
  return (int)std::min<long long>(best, std::max<long long>(1, nfib));
}

// Blocks of the max |T| pass: about 16 KB of T per block, at most 512.
int absmax_blocks(size_t count) {
  return (int)std::max<size_t>(1, std::min<size_t>(512, (count + 4095) / 4096));
}

// Launch shape of a dense build: sketches (bin ranges) per work-group and slabs.
struct BuildPlan {
  int G = 0;
  int nslab = 0;
};

// Bin ranges per sketch: sketches longer than 16384 buckets are split into
// ranges of 16384, one range per work-group (each range reads the whole tensor).
int build_nrange(int b) { return b > 16384 ? b / 16384 : 1; }

// Most sketches one work-group's LDS pool holds (1 with split ranges).
int build_max_g(tsk_tables_t tab) {
  const int nrange = build_nrange(tab->b);
  if (nrange > 1) return 1;
  const size_t per_sketch = (size_t)(tab->b / nrange) * 8;
  return (int)std::min<size_t>({(size_t)tab->B, (size_t)tsk::kBuildMaxG, (size_t)kBuildPoolLarge * 8 / per_sketch});
}

// The rule: as many sketches per work-group as the pool holds; slabs in
// multiples of 8 (one per XCD lane of the grid mapping), as many as fill each
// XCD's 32 CUs in one round (one work-group per CU with the large pool, two
// with the small one), never slabs of fewer than 8 fibres.  G <= 0 asks for the
// largest G.
BuildPlan build_plan_rule(tsk_tables_t tab, int G = 0) {
  const int nrange = build_nrange(tab->b);
  const int Bv = tab->B * nrange;
  const size_t per_sketch = (size_t)(tab->b / nrange) * 8;
  BuildPlan p;
  p.G = G > 0 ? std::min(G, build_max_g(tab)) : build_max_g(tab);
  const int ngroups = (Bv + p.G - 1) / p.G;
  const int Gb = (Bv + ngroups - 1) / ngroups;
  const bool small = (size_t)Gb * per_sketch <= (size_t)kBuildPoolSmall * 8;
  p.nslab = pick_nslab((long long)tab->n * tab->n, ngroups, small);
  return p;
}

template <typename TIn>
tsk_status build_dense_impl(tsk_ctx_t ctx, tsk_tables_t tab, const TIn* T, hipStream_t st,
                            double** s_time_out, BuildPlan plan) {
  const int n = tab->n, b = tab->b, B = tab->B;
  const int nrange = build_nrange(b);
  const int br = b / nrange;
  int lbr = 0;
  while ((1 << lbr) < br) ++lbr;
  const int Bv = B * nrange;                                  // (sketch, range) pairs
  const size_t per_sketch = (size_t)br * 8;  // 64-bit bins
  int G = std::max(1, std::min(plan.G, build_max_g(tab)));
  const int ngroups = (Bv + G - 1) / G;
  G = (Bv + ngroups - 1) / ngroups;  // balance the groups
  const bool small = (size_t)G * per_sketch <= (size_t)kBuildPoolSmall * 8;
  const long long npairs = (long long)n * n;
  // slab lengths are multiples of 4 fibres (the kernel's items)
  int nslab = (int)std::max<long long>(1, std::min<long long>(plan.nslab, npairs));
  long long pps = (npairs + nslab - 1) / nslab;
  pps = (pps + 3) / 4 * 4;
  nslab = (int)((npairs + pps - 1) / pps);
  // Offsets of the first two modes per fibre and sketch: made once per table
  // set, on the first dense build, and complete before that call returns (a
  // later build may run on another stream).
  const long long efs = (npairs + 4 + 3) / 4 * 4;
  if ((size_t)G * efs * 4 > (size_t)0x7fffffff)
    return tsk::fail(TSK_EUNSUPPORTED, "dense build: n=%d too large", n);
  if (!tab->ef) {
    void* d = nullptr;
    TSK_HIP(hipMalloc(&d, (size_t)B * efs * sizeof(uint32_t)));
    hipLaunchKernelGGL(tsk::k_fibre_offsets, dim3(grid_for((size_t)B * efs, 256)), dim3(256), 0, st, tab->hx, n,
                       B, efs, reinterpret_cast<uint32_t*>(d));
    if (check_launch("k_fibre_offsets") != TSK_OK || hipStreamSynchronize(st) != hipSuccess) {
      (void)hipFree(d);
      return tsk::fail(TSK_EHIP, "dense build: fibre offsets failed");
    }
    tab->ef = reinterpret_cast<uint32_t*>(d);
    tab->efs = efs;
  }
  const void* efb = tab->ef;
  void* partial = nullptr;
  void* stime = nullptr;
  void* amax = nullptr;
  TSK_TRY(ws_get(ctx, WS_PARTIAL, (size_t)ngroups * nslab * G * br * sizeof(double), &partial));
  TSK_TRY(ws_get(ctx, WS_STIME, (size_t)B * b * sizeof(double), &stime));
  // per-block max |T| for the fixed-point scale (reduced by the build)
  const size_t cnt = (size_t)n * n * n;
  const int nabs = absmax_blocks(cnt);
  TSK_TRY(ws_get(ctx, WS_AMAX, (size_t)nabs * sizeof(unsigned long long), &amax));
  hipLaunchKernelGGL(tsk::k_absmax<TIn>, dim3(nabs), dim3(256), 0, st, T, cnt,
                     reinterpret_cast<unsigned long long*>(amax));
  TSK_TRY(check_launch("k_absmax"));
  tsk::BuildArgs<TIn> a;
  a.T = T;
  a.n = n;
  a.b = b;
  a.B = B;
  a.G = G;
  a.nrange = nrange;
  a.lbr = lbr;
  a.t3 = tab->hx + 2 * n;
  a.t3s = 3 * n;
  a.ef = reinterpret_cast<const uint32_t*>(efb);
  a.efs = efs;
  a.nfib = npairs;
  a.pairs_per_slab = pps;
  a.nslab = nslab;
  a.ngroups = ngroups;
  a.absmax = reinterpret_cast<const unsigned long long*>(amax);
  a.nabs = nabs;
  a.partial = reinterpret_cast<double*>(partial);
  // 1-D grid: 8 XCD lanes x ngroups x ceil(nslab / 8) (see the kernel).
  const int nblk = 8 * ngroups * ((nslab + 7) / 8);
  TSK_TRY((launch_build<TIn, false>(small, nrange > 1, nblk, a, st)));
  hipLaunchKernelGGL(tsk::k_build_reduce, dim3(grid_for((size_t)B * b, 256)), dim3(256), 0, st,
                     (const double*)partial, (double*)stime, b, B, G, nslab, nrange, lbr);
  TSK_TRY(check_launch("k_build_reduce"));
  *s_time_out = reinterpret_cast<double*>(stime);
  return TSK_OK;
}

}  // namespace

namespace {

std::vector<int> encode_plan(const BuildPlan& p) { return {p.G, p.nslab}; }

// Candidate build plans: every sketches-per-work-group count the pool allows,
// each with the rule's slab count, half of it and twice it; the rule first.
std::vector<BuildPlan> build_candidates(tsk_tables_t tab) {
  std::vector<BuildPlan> out;
  const long long nfib = (long long)tab->n * tab->n;
  for (int G = build_max_g(tab); G >= 1; --G) {
    const BuildPlan r = build_plan_rule(tab, G);
    for (int q : {4, 2, 8}) {
      BuildPlan c;
      c.G = G;
      c.nslab = (int)std::min<long long>(nfib, std::max(8, (r.nslab * q / 4 + 7) / 8 * 8));
      bool dup = false;
      for (const auto& o : out) dup |= (o.G == c.G && o.nslab == c.nslab);
      if (!dup) out.push_back(c);
    }
  }
  return out;
}

template <typename TIn>
tsk_status build_dense_tuned(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, const TIn* T, hipStream_t st,
                             double** stime) {
  BuildPlan plan = build_plan_rule(tab);
  if (ctx->tune_mode != 0) {
    const std::string key = tune_key(ctx, "build", dtype, {tab->n, tab->b, tab->B});
    const std::vector<int>* ch = nullptr;
    auto time_one = [&](const BuildPlan& p, float* ms) -> tsk_status {
      double* scratch_time = nullptr;
      return time_runs(st, 3, [&]() { return build_dense_impl<TIn>(ctx, tab, T, st, &scratch_time, p); }, ms);
    };
    TSK_TRY(tune_choose(ctx, key, build_candidates(tab), encode_plan, time_one, &ch));
    if (ch && ch->size() == 2) {
      plan.G = (*ch)[0];
      plan.nslab = (*ch)[1];
    }
  }
  return build_dense_impl<TIn>(ctx, tab, T, st, stime, plan);
}

}  // namespace

extern "C" tsk_status tsk_sketch_build_dense(tsk_ctx_t ctx, tsk_tables_t tab, const void* T,
                                             tsk_dtype dtype, double* S64, float* S32,
                                             int accumulate, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_sketch_build_dense"));
  if (!T || !S64) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_dense: null T or S64");
  if (dtype != TSK_F32 && dtype != TSK_F64)
    return tsk::fail(TSK_EINVAL, "tsk_sketch_build_dense: bad dtype %d", (int)dtype);
  TSK_TRY(set_device(ctx));
  double* stime = nullptr;
  if (dtype == TSK_F32)
    TSK_TRY(build_dense_tuned<float>(ctx, tab, dtype, (const float*)T, S(stream), &stime));
  else
    TSK_TRY(build_dense_tuned<double>(ctx, tab, dtype, (const double*)T, S(stream), &stime));
  return r2c_any(ctx, tab->logb, stime, reinterpret_cast<cx<double>*>(S64),
                 reinterpret_cast<cx<float>*>(S32), accumulate ? 1 : 0, tab->B, S(stream));
}

extern "C" tsk_status tsk_sketch_from_time(tsk_ctx_t ctx, int b, int B, const double* s_time,
                                           double* S64, float* S32, void* stream) {
  if (!ctx || !s_time || !S64) return tsk::fail(TSK_EINVAL, "tsk_sketch_from_time: null argument");
  const int logb = ilog2_exact(b);
  if (logb < kMinLogB || logb > kMaxLogB || B < 1 || B > 64)
    return tsk::fail(TSK_EINVAL, "tsk_sketch_from_time: b=%d B=%d out of range", b, B);
  TSK_TRY(set_device(ctx));
  return r2c_any(ctx, logb, s_time, reinterpret_cast<cx<double>*>(S64), reinterpret_cast<cx<float>*>(S32), 0,
                 B, S(stream));
}

extern "C" tsk_status tsk_sketch_export(tsk_ctx_t ctx, int b, int B, const double* S64,
                                        double* s_time, void* stream) {
  if (!ctx || !s_time || !S64) return tsk::fail(TSK_EINVAL, "tsk_sketch_export: null argument");
  const int logb = ilog2_exact(b);
  if (logb < kMinLogB || logb > kMaxLogB || B < 1 || B > 64)
    return tsk::fail(TSK_EINVAL, "tsk_sketch_export: b=%d B=%d out of range", b, B);
  TSK_TRY(set_device(ctx));
  return c2r_any(ctx, logb, reinterpret_cast<const cx<double>*>(S64), s_time, B, S(stream));
}

namespace {

// S64 += sign * sum_r lam_r prod_r over `c` vectors U [c][n], in chunks.
tsk_status rank1_update(tsk_ctx_t ctx, tsk_tables_t tab, const double* lam, const double* U, int c,
                        double sign, double* S64, float* S32, hipStream_t st) {
  const int B = tab->B, b = tab->b, n = tab->n;
  const int H1 = b / 2 + 1;
  const cx<double>* tw = nullptr;
  if (tab->logb <= kLdsLogB) TSK_TRY(get_tw<double>(ctx, tab->logb, &tw));
  const size_t per_vec = (size_t)B * H1 * sizeof(cx<double>);
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(16, ((size_t)256 << 20) / per_vec));
  void* prod = nullptr;
  TSK_TRY(ws_get(ctx, WS_PROD, (size_t)std::min(chunk, c) * per_vec, &prod));
  void* ebuf = nullptr;
  if (rank1_split_path(tab->logb))
    TSK_TRY(ws_get(ctx, WS_SPLITP, rank1_split_bytes(tab, std::min(chunk, c)), &ebuf));
  for (int r0 = 0; r0 < c; r0 += chunk) {
    const int cc = std::min(chunk, c - r0);
    tsk::Rank1Args a;
    a.hx = tab->hx;
    a.hxs = tab->hxs;
    a.ord = tab->ord;
    a.n = n;
    a.B = B;
    a.U = U + (size_t)r0 * n;
    a.twg = tw;
    a.prod = reinterpret_cast<cx<double>*>(prod);
    a.S64 = nullptr;
    a.lam_per = nullptr;
    TSK_TRY(launch_rank1_any(ctx, tab, a, cc, ebuf, st));
    hipLaunchKernelGGL(tsk::k_spec_update, dim3(grid_for((size_t)B * H1, 256)), dim3(256), 0, st,
                       reinterpret_cast<cx<double>*>(S64), reinterpret_cast<cx<float>*>(S32),
                       (const cx<double>*)prod, lam + r0, sign, cc, B, H1);
    TSK_TRY(check_launch("k_spec_update"));
  }
  return TSK_OK;
}

}  // namespace

extern "C" tsk_status tsk_sketch_build_factors(tsk_ctx_t ctx, tsk_tables_t tab, const double* lam,
                                               const double* A, int k, double* S64, float* S32,
                                               int accumulate, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_sketch_build_factors"));
  if (!lam || !A || !S64) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_factors: null argument");
  if (k < 1) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_factors: k=%d < 1", k);
  TSK_TRY(set_device(ctx));
  const size_t H1 = (size_t)tab->b / 2 + 1;
  if (!accumulate) {
    const size_t words = (size_t)tab->B * H1 * 4;  // doubles as u32 pairs
    hipLaunchKernelGGL(tsk::k_fill_u32, dim3(grid_for(words, 256)), dim3(256), 0, S(stream),
                       reinterpret_cast<unsigned*>(S64), 0u, words);
    TSK_TRY(check_launch("k_fill_u32"));
  }
  return rank1_update(ctx, tab, lam, A, k, +1.0, S64, S32, S(stream));
}

extern "C" tsk_status tsk_sketch_deflate(tsk_ctx_t ctx, tsk_tables_t tab, const double* lam,
                                         const double* U, int c, double* S64, float* S32,
                                         void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_sketch_deflate"));
  if (!lam || !U || !S64) return tsk::fail(TSK_EINVAL, "tsk_sketch_deflate: null argument");
  if (c < 1) return tsk::fail(TSK_EINVAL, "tsk_sketch_deflate: c=%d < 1", c);
  TSK_TRY(set_device(ctx));
  return rank1_update(ctx, tab, lam, U, c, -1.0, S64, S32, S(stream));
}

// =============================================================================
// Contractions
// =============================================================================

namespace {


// FP32 power step at b = 65536 through the split transforms (large.hpp), one
// launch (k_power_split1).  The median of the previous step (prefix) is the
// kernel's prologue when u fits the LDS beside the buffer and B <= 16 (the
// sorting-network median); otherwise a launch of its own before the step.
// n whose u fits the LDS beside the M-point buffer
constexpr int kSplit1MaxULds = (int)((kMaxLds - tsk::split1_lds_bytes(kSubLogM32, 0, false)) / sizeof(float));

tsk_status power_split(tsk_ctx_t ctx, tsk_tables_t tab, const cx<float>* spec, int nrest, int tau0,
                       int prefix, int mode, const float* Uprev, const float* Vprev, float* Ucur,
                       int32_t* flags, float* V, double* lam_per, hipStream_t st, int perm,
                       const SplitBufs* sb, const float* Uy = nullptr) {
  if (!sb || !sb->A) return tsk::fail(TSK_EHIP, "internal: split power buffers missing");
  const int n = tab->n, B = tab->B;
  const cx<float>* twM = nullptr;
  const cx<float>* Wb = nullptr;
  TSK_TRY(get_tw<float>(ctx, kSubLogM32 + 1, &twM, tsk::kSplit1Threads));
  TSK_TRY(get_wb<float>(ctx, tab->logb, &Wb));
  const bool u_lds = n <= kSplit1MaxULds;
  const bool pre = prefix && u_lds && B <= 16;
  if (prefix && !pre) {
    const size_t on = (size_t)tau0 * n, obn = (size_t)tau0 * B * n;
    TSK_TRY(median_norm_launch<float>(Vprev + obn, Uprev + on, Ucur + on, flags ? flags + tau0 : nullptr,
                                      nrest, n, B, st));
    Uprev = Ucur;
  }
  tsk::SplitOneArgs a;
  a.hx = tab->hx;
  a.hxs = tab->hxs;
  a.ord = tab->ord;
  a.n = n;
  a.B = B;
  a.S = spec;
  a.Wb = Wb;
  a.twM = twM;
  a.Uprev = Uprev;
  a.Uy = Uy;
  a.Vprev = Vprev;
  a.Ucur = Ucur;
  a.flags = flags;
  a.V = V;
  a.lam_per = lam_per;
  a.P = reinterpret_cast<cx<float>*>(sb->A);
  a.tau0 = tau0;
  a.mode = mode;
  a.u_lds = u_lds ? 1 : 0;
  a.rd = perm;
  a.sa = (perm + 1) % 3;
  a.sb = (perm + 2) % 3;
  const size_t lds = tsk::split1_lds_bytes(kSubLogM32, n, u_lds);
  const int dev = ctx->device;
  static std::atomic<uint64_t> configured{0};
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_power_split1<kSubLogM32, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_power_split1<kSubLogM32, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    configured.fetch_or(bit);
  }
  if (pre)
    hipLaunchKernelGGL((tsk::k_power_split1<kSubLogM32, true>), dim3(B, nrest), dim3(tsk::kSplit1Threads), lds,
                       st, a);
  else
    hipLaunchKernelGGL((tsk::k_power_split1<kSubLogM32, false>), dim3(B, nrest), dim3(tsk::kSplit1Threads), lds,
                       st, a);
  return check_launch("k_power_split1");
}

template <typename R>
tsk_status power_launch(tsk_ctx_t ctx, tsk_tables_t tab, const void* spec, int nrest, int tau0,
                        int prefix, int mode, const R* Uprev, const R* Vprev, R* Ucur,
                        int32_t* flags, R* V, double* lam_per, hipStream_t st, int perm = 0,
                        const SplitBufs* sb = nullptr, const R* Uy = nullptr) {
  if (tab->logb > kLdsLogB + 1 || (sizeof(R) == 8 && tab->logb > kLdsLogB)) {
    if constexpr (sizeof(R) == 4)
      return power_split(ctx, tab, reinterpret_cast<const cx<float>*>(spec), nrest, tau0, prefix, mode, Uprev,
                         Vprev, Ucur, flags, V, lam_per, st, perm, sb, Uy);
    return tsk::fail(TSK_EUNSUPPORTED, "power step: FP64 supports b <= 16384 (b=%d)", tab->b);
  }
  const cx<R>* tw = nullptr;
  TSK_TRY(get_tw<R>(ctx, tab->logb, &tw));
  tsk::PowerArgs<R> a;
  a.hx = tab->hx;
  a.hxs = tab->hxs;
  a.ord = tab->ord;
  a.n = tab->n;
  a.B = tab->B;
  a.S = reinterpret_cast<const cx<R>*>(spec);
  a.twg = tw;
  a.Uprev = Uprev;
  a.Uy = Uy;
  a.Vprev = Vprev;
  a.Ucur = Ucur;
  a.flags = flags;
  a.V = V;
  a.lam_per = lam_per;
  a.tau0 = tau0;
  a.prefix = prefix;
  a.mode = mode;
  a.tab_lds = 0;
  a.rd = perm;
  a.sa = (perm + 1) % 3;
  a.sb = (perm + 2) % 3;
  return launch_power<R>(tab->logb, a, tab->B, nrest, st);
}

// Buffers for an eager (uncaptured) call on nvec vectors.
tsk_status eager_split_bufs(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, int nvec, SplitBufs* sb) {
  if (!needs_power_split(tab, dtype)) return TSK_OK;
  void* p = nullptr;
  TSK_TRY(ws_get(ctx, WS_SPLIT, power_split_bytes_A(tab, nvec), &p));
  sb->A = p;
  return TSK_OK;
}

tsk_status lam_median_launch(const double* lam_per, double* lam_med, int L, int B, hipStream_t st) {
  hipLaunchKernelGGL(tsk::k_lam_median, dim3((L + 3) / 4), dim3(256), 0, st, lam_per, lam_med, L, B);
  return check_launch("k_lam_median");
}

tsk_status check_power_args(tsk_tables_t tab, tsk_dtype dtype, const double* S64, const float* S32,
                            int L, const char* fn) {
  if (dtype != TSK_F32 && dtype != TSK_F64) return tsk::fail(TSK_EINVAL, "%s: bad dtype", fn);
  if (L < 1) return tsk::fail(TSK_EINVAL, "%s: L=%d < 1", fn, L);
  if (dtype == TSK_F32 && !S32) return tsk::fail(TSK_EINVAL, "%s: FP32 path needs S32", fn);
  if (dtype == TSK_F64 && !S64) return tsk::fail(TSK_EINVAL, "%s: FP64 path needs S64", fn);
  if (dtype == TSK_F64 && tab->logb > kLdsLogB)
    return tsk::fail(TSK_EUNSUPPORTED, "%s: FP64 power steps support b <= 16384 (b=%d)", fn, tab->b);
  if (L > 65535) return tsk::fail(TSK_EINVAL, "%s: L=%d > 65535", fn, L);
  return TSK_OK;
}

}  // namespace

extern "C" tsk_status tsk_power_update(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                       const double* S64, const float* S32, int L,
                                       const void* U_in, void* U_out, void* V, int32_t* flags,
                                       void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_power_update"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, "tsk_power_update"));
  if (!U_in || !U_out) return tsk::fail(TSK_EINVAL, "tsk_power_update: null vector buffer");
  if (U_in == U_out) return tsk::fail(TSK_EINVAL, "tsk_power_update: U_in and U_out alias");
  TSK_TRY(set_device(ctx));
  const size_t es = dtype == TSK_F32 ? 4 : 8;
  void* vbuf = V;
  if (!vbuf) TSK_TRY(ws_get(ctx, WS_V, (size_t)L * tab->B * tab->n * es, &vbuf));
  const int n = tab->n, B = tab->B;
  SplitBufs sb;
  TSK_TRY(eager_split_bufs(ctx, tab, dtype, L, &sb));
  if (dtype == TSK_F32) {
    TSK_TRY(power_launch<float>(ctx, tab, S32, L, 0, 0, 0, (const float*)U_in, nullptr, nullptr,
                                nullptr, (float*)vbuf, nullptr, S(stream), 0, &sb));
    return median_norm_launch<float>((const float*)vbuf, (const float*)U_in, (float*)U_out, flags, L,
                                     n, B, S(stream));
  }
  TSK_TRY(power_launch<double>(ctx, tab, S64, L, 0, 0, 0, (const double*)U_in, nullptr, nullptr,
                               nullptr, (double*)vbuf, nullptr, S(stream)));
  return median_norm_launch<double>((const double*)vbuf, (const double*)U_in, (double*)U_out, flags,
                                    L, n, B, S(stream));
}

extern "C" tsk_status tsk_power_update_noalloc(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                               const double* S64, const float* S32, int L,
                                               const void* U_in, void* U_out, int32_t* flags,
                                               void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_power_update_noalloc"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, "tsk_power_update_noalloc"));
  if (!U_in || !U_out) return tsk::fail(TSK_EINVAL, "tsk_power_update_noalloc: null vector buffer");
  if (U_in == U_out) return tsk::fail(TSK_EINVAL, "tsk_power_update_noalloc: U_in and U_out alias");
  if (!ctx->scratch) return tsk::fail(TSK_EHIP, "tsk_power_update_noalloc: no scratch address");
  const int n = tab->n, B = tab->B;
  const size_t es = dtype == TSK_F32 ? 4 : 8;
  const size_t vbytes = ((size_t)L * B * n * es + 255) & ~(size_t)255;
  const size_t abytes = needs_power_split(tab, dtype) ? power_split_bytes_A(tab, L) : 0;
  const size_t need = vbytes + abytes;
  if (need > kScratchBytes)
    return tsk::fail(TSK_EINVAL,
                     "tsk_power_update_noalloc: L=%d, B=%d, n=%d, b=%d needs %zu bytes of scratch, more than "
                     "its %zu; take fewer vectors per call or use tsk_power_update",
                     L, B, n, tab->b, need, kScratchBytes);
  TSK_TRY(set_device(ctx));
  NoAllocGuard guard(ctx);
  char* base = reinterpret_cast<char*>(ctx->scratch);
  void* vbuf = base;
  SplitBufs sb;
  if (abytes) sb.A = base + vbytes;
  if (dtype == TSK_F32) {
    TSK_TRY(power_launch<float>(ctx, tab, S32, L, 0, 0, 0, (const float*)U_in, nullptr, nullptr,
                                nullptr, (float*)vbuf, nullptr, S(stream), 0, &sb));
    return median_norm_launch<float>((const float*)vbuf, (const float*)U_in, (float*)U_out, flags, L,
                                     n, B, S(stream));
  }
  TSK_TRY(power_launch<double>(ctx, tab, S64, L, 0, 0, 0, (const double*)U_in, nullptr, nullptr,
                               nullptr, (double*)vbuf, nullptr, S(stream)));
  return median_norm_launch<double>((const double*)vbuf, (const double*)U_in, (double*)U_out, flags,
                                    L, n, B, S(stream));
}

extern "C" tsk_status tsk_median_normalize(tsk_ctx_t ctx, tsk_dtype dtype, int L, int n, int B,
                                           const void* V, const void* U_in, void* U_out,
                                           int32_t* flags, void* stream) {
  if (!ctx || !V || !U_in || !U_out)
    return tsk::fail(TSK_EINVAL, "tsk_median_normalize: null argument");
  if (L < 1 || n < 1 || B < 1)
    return tsk::fail(TSK_EINVAL, "tsk_median_normalize: L=%d, n=%d, B=%d must be >= 1", L, n, B);
  if (dtype != TSK_F32 && dtype != TSK_F64)
    return tsk::fail(TSK_EINVAL, "tsk_median_normalize: dtype %d", (int)dtype);
  if (U_out == V || U_out == U_in)
    return tsk::fail(TSK_EINVAL, "tsk_median_normalize: U_out aliases V or U_in");
  TSK_TRY(set_device(ctx));
  if (dtype == TSK_F32)
    return median_norm_launch<float>((const float*)V, (const float*)U_in, (float*)U_out, flags, L, n, B,
                                     S(stream));
  return median_norm_launch<double>((const double*)V, (const double*)U_in, (double*)U_out, flags, L, n,
                                    B, S(stream));
}

extern "C" tsk_status tsk_contract_tiuu(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                        const double* S64, const float* S32, int L, const void* U,
                                        void* V, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_contract_tiuu"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, "tsk_contract_tiuu"));
  if (!U || !V) return tsk::fail(TSK_EINVAL, "tsk_contract_tiuu: null U or V");
  TSK_TRY(set_device(ctx));
  SplitBufs sb;
  TSK_TRY(eager_split_bufs(ctx, tab, dtype, L, &sb));
  if (dtype == TSK_F32)
    return power_launch<float>(ctx, tab, S32, L, 0, 0, 0, (const float*)U, nullptr, nullptr, nullptr,
                               (float*)V, nullptr, S(stream), 0, &sb);
  return power_launch<double>(ctx, tab, S64, L, 0, 0, 0, (const double*)U, nullptr, nullptr, nullptr,
                              (double*)V, nullptr, S(stream));
}

extern "C" tsk_status tsk_contract_two(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                       const double* S64, const float* S32, int rd, int L,
                                       const void* X, const void* Y, void* V, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_contract_two"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, "tsk_contract_two"));
  if (!X || !Y || !V) return tsk::fail(TSK_EINVAL, "tsk_contract_two: null X, Y or V");
  if (rd < 0 || rd > 2) return tsk::fail(TSK_EINVAL, "tsk_contract_two: rd=%d outside [0,2]", rd);
  TSK_TRY(set_device(ctx));
  SplitBufs sb;
  TSK_TRY(eager_split_bufs(ctx, tab, dtype, L, &sb));
  if (dtype == TSK_F32)
    return power_launch<float>(ctx, tab, S32, L, 0, 0, 0, (const float*)X, nullptr, nullptr, nullptr,
                               (float*)V, nullptr, S(stream), rd, &sb, (const float*)Y);
  return power_launch<double>(ctx, tab, S64, L, 0, 0, 0, (const double*)X, nullptr, nullptr, nullptr,
                              (double*)V, nullptr, S(stream), rd, nullptr, (const double*)Y);
}

namespace {

// Algorithm 2 for k factors: T sweeps of the A, B, C updates.
template <typename R>
tsk_status als_enqueue(tsk_ctx_t ctx, tsk_tables_t tab, const void* spec, int k, int T, double* lam_out,
                       double* F, char* ws, const SplitBufs* sb, hipStream_t st) {
  const int n = tab->n, B = tab->B;
  const size_t kn = (size_t)k * n;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = ws + off;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  R* Fr = (R*)take(3 * kn * sizeof(R));
  R* V = (R*)take(kn * B * sizeof(R));
  double* Vbar = (double*)take(kn * 8);
  double* G = (double*)take((size_t)k * k * 8);
  double* P = (double*)take((size_t)k * k * 8);
  hipLaunchKernelGGL(tsk::k_cvt<R>, dim3(grid_for(3 * kn, 256)), dim3(256), 0, st, (const double*)F, Fr,
                     3 * kn);
  TSK_TRY(check_launch("k_cvt"));
  for (int t = 0; t < T; ++t) {
    for (int rd = 0; rd < 3; ++rd) {
      const int ix = (rd + 1) % 3, iy = (rd + 2) % 3;
      TSK_TRY(power_launch<R>(ctx, tab, spec, k, 0, 0, 0, Fr + ix * kn, nullptr, nullptr, nullptr, V,
                              nullptr, st, rd, sb, Fr + iy * kn));
      hipLaunchKernelGGL(tsk::k_median_rows<R>, dim3(k), dim3(tsk::median_threads<R>()), 0, st,
                         (const R*)V, Vbar, n, B);
      TSK_TRY(check_launch("k_median_rows"));
      hipLaunchKernelGGL(tsk::k_als_gram, dim3(k, k), dim3(256), 0, st, (const double*)(F + ix * kn),
                         (const double*)(F + iy * kn), G, n, k);
      TSK_TRY(check_launch("k_als_gram"));
      hipLaunchKernelGGL(tsk::k_als_pinv, dim3(1), dim3(256), 0, st, (const double*)G, P, k);
      TSK_TRY(check_launch("k_als_pinv"));
      hipLaunchKernelGGL(tsk::k_als_apply, dim3((n + 255) / 256, k), dim3(256), 0, st, (const double*)P,
                         (const double*)Vbar, F + rd * kn, n, k);
      TSK_TRY(check_launch("k_als_apply"));
      hipLaunchKernelGGL(tsk::k_als_normalize<R>, dim3(k), dim3(256), 0, st, F + rd * kn, Fr + rd * kn,
                         lam_out, n);
      TSK_TRY(check_launch("k_als_normalize"));
    }
  }
  return TSK_OK;
}

size_t als_ws_bytes(tsk_tables_t tab, tsk_dtype dtype, int k) {
  const size_t kn = (size_t)k * tab->n, es = dtype == TSK_F32 ? 4 : 8;
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  return r(3 * kn * es) + r(kn * tab->B * es) + r(kn * 8) + 2 * r((size_t)k * k * 8);
}

}  // namespace

extern "C" tsk_status tsk_als(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, const double* S64,
                              const float* S32, int k, int T, const double* F0, double* lam_out,
                              double* F_out, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_als"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, k, "tsk_als"));
  if (!F0 || !lam_out || !F_out) return tsk::fail(TSK_EINVAL, "tsk_als: null F0, lam_out or F_out");
  if (k < 1 || k > 64) return tsk::fail(TSK_EINVAL, "tsk_als: k=%d outside [1,64]", k);
  if (T < 1) return tsk::fail(TSK_EINVAL, "tsk_als: T=%d < 1", T);
  if (dtype == TSK_F64 && tab->logb > kLdsLogB)
    return tsk::fail(TSK_EUNSUPPORTED, "tsk_als: FP64 power steps support b <= 16384 (b=%d)", tab->b);
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  void* ws = nullptr;
  TSK_TRY(ws_get(ctx, WS_ALS, als_ws_bytes(tab, dtype, k), &ws));
  SplitBufs sb;
  TSK_TRY(eager_split_bufs(ctx, tab, dtype, k, &sb));
  if (F_out != F0)
    TSK_HIP(hipMemcpyAsync(F_out, F0, (size_t)3 * k * tab->n * 8, hipMemcpyDeviceToDevice, st));
  if (dtype == TSK_F32)
    return als_enqueue<float>(ctx, tab, S32, k, T, lam_out, F_out, (char*)ws, &sb, st);
  return als_enqueue<double>(ctx, tab, S64, k, T, lam_out, F_out, (char*)ws, &sb, st);
}

extern "C" tsk_status tsk_contract_uuu(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                       const double* S64, const float* S32, int L, const void* U,
                                       double* lam_med, double* lam_per, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_contract_uuu"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, "tsk_contract_uuu"));
  if (!U || !lam_med) return tsk::fail(TSK_EINVAL, "tsk_contract_uuu: null U or lam_med");
  TSK_TRY(set_device(ctx));
  const size_t es = dtype == TSK_F32 ? 4 : 8;
  void* vbuf = nullptr;
  TSK_TRY(ws_get(ctx, WS_V, (size_t)L * tab->B * tab->n * es, &vbuf));
  void* lp = lam_per;
  if (!lp) TSK_TRY(ws_get(ctx, WS_LAMPER, (size_t)L * tab->B * sizeof(double), &lp));
  SplitBufs sb;
  TSK_TRY(eager_split_bufs(ctx, tab, dtype, L, &sb));
  if (dtype == TSK_F32)
    TSK_TRY(power_launch<float>(ctx, tab, S32, L, 0, 0, 1, (const float*)U, nullptr, nullptr,
                                nullptr, (float*)vbuf, (double*)lp, S(stream), 0, &sb));
  else
    TSK_TRY(power_launch<double>(ctx, tab, S64, L, 0, 0, 1, (const double*)U, nullptr, nullptr,
                                 nullptr, (double*)vbuf, (double*)lp, S(stream)));
  return lam_median_launch((const double*)lp, lam_med, L, tab->B, S(stream));
}

// =============================================================================
// Sketch of the whitened LDA moment from document word counts (Appendix D)
// =============================================================================

namespace {

template <typename R>
size_t terms_lds_bytes(int logh, int n) {
  const size_t PL = (size_t)tsk::padded_len(1 << logh);
  return tsk::align16(sizeof(R) * 2 * PL) + 2 * sizeof(R) * (size_t)((n + 3) & ~3) + 24 * (size_t)n;
}

template <typename R, int LOGB, bool HAS_Y>
tsk_status launch_terms_t(const tsk::TermArgs& a, int B, int nchunk, hipStream_t st) {
  // the word terms hold three running products: their bins go in two rounds
  constexpr int NPART = HAS_Y ? 2 : 1;
  constexpr int NT = tsk::threads_for_h<R>(LOGB - 1);
  const size_t lds = terms_lds_bytes<R>(LOGB - 1, a.n);
  if (lds > kMaxLds)
    return tsk::fail(TSK_EUNSUPPORTED, "document sketch: K=%d needs %zu bytes of LDS at b=2^%d", a.n, lds,
                     LOGB);
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_terms<R, LOGB, HAS_Y, NPART>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL((tsk::k_terms<R, LOGB, HAS_Y, NPART>), dim3(B, nchunk), dim3(NT), lds, st, a);
  return check_launch("k_terms");
}

template <typename R, bool HAS_Y>
tsk_status launch_terms(int logb, const tsk::TermArgs& a, int B, int nchunk, hipStream_t st) {
#define TSK_TERMS(L) launch_terms_t<R, L, HAS_Y>(a, B, nchunk, st)
  TSK_LOGB_SWITCH(logb, TSK_TERMS);
#undef TSK_TERMS
  return tsk::fail(TSK_EUNSUPPORTED, "document sketch: b=2^%d not built", logb);
}

template <typename R, int LOGB>
tsk_status launch_mode_spectra_t(tsk_tables_t tab, const double* q, const cx<R>* tw, cx<R>* Qs,
                                 hipStream_t st) {
  hipLaunchKernelGGL((tsk::k_mode_spectra<R, LOGB>), dim3(tab->B, 3), dim3(tsk::threads_for_h<R>(LOGB - 1)),
                     0, st, tab->hxs, tab->ord, tab->n, q, tw, Qs);
  return check_launch("k_mode_spectra");
}

template <typename R>
tsk_status launch_mode_spectra(int logb, tsk_tables_t tab, const double* q, const cx<R>* tw, cx<R>* Qs,
                               hipStream_t st) {
#define TSK_MSPEC(L) launch_mode_spectra_t<R, L>(tab, q, tw, Qs, st)
  TSK_LOGB_SWITCH(logb, TSK_MSPEC);
#undef TSK_MSPEC
  return tsk::fail(TSK_EUNSUPPORTED, "document sketch: b=2^%d not built", logb);
}

// G = X^T Y for X, Y: [V][K] in FP64: 16 x 16 tiles over word chunks (about
// 512 words each, at most 32), the chunks' partials summed in chunk order.
tsk_status gram2(tsk_ctx_t ctx, const double* X, const double* Y, double* G, int V, int K, hipStream_t st) {
  const int nt = (K + 15) / 16;
  const int Z = std::max(1, std::min(32, V / 512));
  void* part = nullptr;
  TSK_TRY(ws_get(ctx, WS_GRAM, (size_t)Z * K * K * sizeof(double), &part));
  hipLaunchKernelGGL(tsk::k_gram2, dim3(nt, nt, Z), dim3(256), 0, st, X, Y, (double*)part, V, K, Z);
  TSK_TRY(check_launch("k_gram2"));
  hipLaunchKernelGGL(tsk::k_gram2_sum, dim3(grid_for((size_t)K * K, 256)), dim3(256), 0, st, (const double*)part,
                     Z, K, G);
  return check_launch("k_gram2_sum");
}

// Bit width of the word ids 0..V-1: the radix sort by word reads only those bits.
int word_bits(int V) {
  int b = 1;
  while (b < 31 && (1 << b) < V) ++b;
  return b;
}

// Temporary storage of the stable sort of the nonzeros by word.
hipError_t word_sort_tmp(size_t* bytes, int nnz, int V, hipStream_t st) {
  return rocprim::radix_sort_pairs(nullptr, *bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                   (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                   (size_t)std::max(nnz, 1), 0, word_bits(V), st);
}

// The nonzeros in word order, stable in document order: the sorted word ids
// skeys, the first position of every word colptr[V+1], and the document and
// count of each nonzero (sdoc, scnt).  pin, pout: 8 nnz bytes each; scnt may
// share pin's memory (pin is free once the sort has read it).
tsk_status word_order(const int32_t* rowptr, const int32_t* col, const int32_t* cnt, int D, int V, int nnz,
                      unsigned long long* pin, unsigned long long* pout, uint32_t* skeys, void* tmp,
                      size_t tmp_bytes, int32_t* colptr, int32_t* sdoc, int32_t* scnt, hipStream_t st) {
  if (nnz > 0) {
    hipLaunchKernelGGL(tsk::k_pack_entries, dim3(std::min((D + 3) / 4, 65536)), dim3(256), 0, st, rowptr, cnt, D,
                       pin);
    TSK_TRY(check_launch("k_pack_entries"));
    size_t t = tmp_bytes;
    TSK_HIP(rocprim::radix_sort_pairs(tmp, t, reinterpret_cast<const uint32_t*>(col), skeys,
                                      (const unsigned long long*)pin, pout, (size_t)nnz, 0, word_bits(V), st));
  }
  hipLaunchKernelGGL(tsk::k_col_bounds, dim3(grid_for((size_t)V + 1, 256)), dim3(256), 0, st,
                     reinterpret_cast<const int32_t*>(skeys), nnz, V, colptr);
  TSK_TRY(check_launch("k_col_bounds"));
  if (nnz > 0) {
    hipLaunchKernelGGL(tsk::k_unpack_entries, dim3(grid_for((size_t)nnz, 256)), dim3(256), 0, st,
                       (const unsigned long long*)pout, nnz, sdoc, scnt);
    TSK_TRY(check_launch("k_unpack_entries"));
  }
  return TSK_OK;
}

// Shapes of the moment route's products: the pair rows padded to whole
// work-group blocks, the column groups, and the item chunks.  A wave leaves
// out the column tiles below its rows' smallest b, so the work of a row block
// falls with b; about four rounds of work-groups over two per CU let the
// dispatcher even that out (the chunk partials are capped at 256 MB).
struct MomentShape {
  int np = 0, rows = 0, nrb = 0;
  int ncg_d = 0, ld_d = 0, nch_d = 0, per_d = 0;
  int ncg_w = 0, ld_w = 0, nch_w = 0, per_w = 0;
  size_t part_bytes_d = 0, part_bytes_w = 0;
};

MomentShape moment_shape(int K, int D, int V) {
  MomentShape m;
  m.np = K * (K + 1) / 2;
  m.nrb = (m.np + tsk::kMomRows - 1) / tsk::kMomRows;
  m.rows = m.nrb * tsk::kMomRows;
  auto cols = [&](int ncol, int nitem, int& ncg, int& ld, int& nch, int& per) {
    ncg = (ncol + tsk::kMomCols - 1) / tsk::kMomCols;
    ld = ncg * tsk::kMomCols;
    const int wgs = m.nrb * ncg;
    const size_t chunk_bytes = (size_t)m.rows * ld * sizeof(double);
    nch = std::max(1, std::min(64, 4 * 512 / wgs));
    nch = std::max(1, std::min<int>(nch, (int)((256u << 20) / chunk_bytes)));
    nch = std::max(1, std::min(nch, (nitem + 255) / 256));  // at least 256 items per chunk
    per = (nitem + nch - 1) / nch;
    per = (per + 3) & ~3;
    nch = std::max(1, (nitem + per - 1) / per);
  };
  cols(K + 1, D, m.ncg_d, m.ld_d, m.nch_d, m.per_d);
  cols(2 * K + 1, V, m.ncg_w, m.ld_w, m.nch_w, m.per_w);
  m.part_bytes_d = (size_t)m.nch_d * m.rows * m.ld_d * sizeof(double);
  m.part_bytes_w = (size_t)m.nch_w * m.rows * m.ld_w * sizeof(double);
  return m;
}

// Route of the document build: the moment tensor when its matrix-core work
// (FP64, about 15 TFLOP/s measured on the useful multiply-adds) is estimated
// below the per-document transforms (2.5 b log2 b flops per real transform,
// about 16 TFLOP/s measured in FP32, 6 in FP64, on the vector units);
// tsk_docs_route overrides the rule.
bool docs_use_moment(const tsk_ctx* ctx, int K, int B, int b, int D, int V, bool fp64) {
  if (ctx->docs_route == 1) return false;
  if (ctx->docs_route == 2) return true;
  // about K^3 / 6 + K^2 / 2 multiply-adds per document (the x^(x)3 columns at
  // c >= b, the second-order column) and K^3 / 6 + K^3 / 2 + K^2 / 2 per word
  const double k3 = (double)K * K * K, k2 = (double)K * K;
  const double mflop = 2.0 * ((k3 / 6 + k2 / 2) * D + (2 * k3 / 3 + k2 / 2) * V);
  const double tflop = (3.0 * D + 6.0 * V) * B * 2.5 * b * std::log2((double)b);
  return mflop / 15e12 < tflop / (fp64 ? 6e12 : 16e12);
}

// One product of the moment route (documents, or words with HAS_Y) and the
// sum of its chunks into C [np][ncol].
template <typename R, bool HAS_Y>
tsk_status launch_moment(const MomentShape& ms, const R* X, const R* Y, const double* cA, const double* cB,
                         double sa, double sb, double gam, int K, int nitem, double* part, double* C,
                         hipStream_t st) {
  tsk::MomentArgs m;
  m.X = X;
  m.Y = Y;
  m.cA = cA;
  m.cB = cB;
  m.sa = sa;
  m.sb = sb;
  m.gam = gam;
  m.K = K;
  m.nitem = nitem;
  m.per = HAS_Y ? ms.per_w : ms.per_d;
  m.np = ms.np;
  m.ncol = HAS_Y ? 2 * K + 1 : K + 1;
  m.rows = ms.rows;
  m.ld = HAS_Y ? ms.ld_w : ms.ld_d;
  m.part = part;
  const int ncg = HAS_Y ? ms.ncg_w : ms.ncg_d, nch = HAS_Y ? ms.nch_w : ms.nch_d;
  const size_t lds = tsk::moment_lds_bytes(K, HAS_Y);
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_moment3<R, HAS_Y>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)tsk::moment_lds_bytes(128, true)));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL((tsk::k_moment3<R, HAS_Y>), dim3(ms.nrb * ncg, nch), dim3(256), lds, st, m);
  TSK_TRY(check_launch("k_moment3"));
  hipLaunchKernelGGL(tsk::k_moment_reduce, dim3(grid_for((size_t)ms.np * m.ncol, 256)), dim3(256), 0, st,
                     (const double*)part, nch, ms.rows, m.ld, ms.np, m.ncol, C);
  return check_launch("k_moment_reduce");
}

template <typename R>
tsk_status build_docs_impl(tsk_ctx_t ctx, tsk_tables_t tab, const int32_t* rowptr, const int32_t* col,
                           const int32_t* cnt, int D, int V, int nnz, const R* W, double alpha0,
                           double* S64, float* S32, int accumulate, hipStream_t st) {
  const int K = tab->n, B = tab->B, b = tab->b, logb = tab->logb;
  const int H1 = b / 2 + 1;
  const cx<R>* tw = nullptr;  // the document kernels run threads_for_h threads
  TSK_TRY(get_tw<R>(ctx, logb, &tw, tsk::threads_for_h<R>(logb - 1)));
  const int G = std::max(1, std::min(1024, (D + 255) / 256));
  const int per_q = (D + G - 1) / G;
  const int ncD = std::max(1, std::min(128, (D + 63) / 64));
  const int ncW = std::max(1, std::min(64, (V + 63) / 64));
  size_t sort_tmp = 0;
  TSK_HIP(word_sort_tmp(&sort_tmp, nnz, V, st));
  // one workspace, 256-byte aligned pieces
  size_t off = 0;
  std::vector<size_t> offs;
  auto take = [&](size_t bytes) {
    offs.push_back(off);
    off += (bytes + 255) & ~(size_t)255;
  };
  take((size_t)D * K * sizeof(R));              // 0 P
  take((size_t)D * 8);                          // 1 cd
  take((size_t)D * 8);                          // 2 cpd
  take((size_t)D * 8);                          // 3 invm
  take((size_t)G * (K + 1) * 8);                // 4 q partials
  take((size_t)K * 8);                          // 5 q
  take(8);                                      // 6 D_eff
  take((size_t)nnz * 8);                        // 7 packed entries (then the counts in word order)
  take((size_t)nnz * 8);                        // 8 packed entries in word order
  take((size_t)nnz * 4);                        // 9 sorted word ids
  take((size_t)nnz * 4);                        // 10 documents in word order
  take(sort_tmp);                               // 11 sort scratch
  take((size_t)(V + 1) * 4);                    // 12 colptr
  take((size_t)V * K * sizeof(R));              // 13 R_i
  take((size_t)V * 8);                          // 14 g
  take((size_t)V * 8);                          // 15 g'
  const bool moment = docs_use_moment(ctx, K, B, b, D, V, sizeof(R) == 8);
  const MomentShape ms = moment_shape(K, D, V);
  take(moment ? 0 : (size_t)B * 3 * H1 * sizeof(cx<R>));   // 16 Q spectra
  take(moment ? 0 : (size_t)B * ncD * H1 * 16);            // 17 document partials
  take(moment ? 0 : (size_t)B * ncW * H1 * 16);            // 18 word partials
  take(moment ? ms.part_bytes_d : 0);                       // 19 document products per chunk
  take(moment ? ms.part_bytes_w : 0);                       // 20 word products per chunk
  take(moment ? (size_t)ms.np * (K + 1) * 8 : 0);           // 21 Cd
  take(moment ? (size_t)ms.np * (2 * K + 1) * 8 : 0);       // 22 Cw
  take(moment ? (size_t)K * K * K * 8 : 0);                 // 23 the K^3 tensor
  take((size_t)D * 16);                                     // 24 packed (cd, cpd) per document
  void* base = nullptr;
  TSK_TRY(ws_get(ctx, WS_DOCS, off, &base));
  auto at = [&](int i) { return reinterpret_cast<char*>(base) + offs[i]; };
  R* P = (R*)at(0);
  double *cd = (double*)at(1), *cpd = (double*)at(2), *invm = (double*)at(3);
  double *qpart = (double*)at(4), *q = (double*)at(5), *deff = (double*)at(6);
  int32_t* colptr = (int32_t*)at(12);
  R* Rw = (R*)at(13);
  double *g = (double*)at(14), *gp = (double*)at(15);
  cx<R>* Qs = (cx<R>*)at(16);
  cx<double>* partD = (cx<double>*)at(17);
  cx<double>* partW = (cx<double>*)at(18);

  hipLaunchKernelGGL(tsk::k_doc_project<R>, dim3(std::min((D + 15) / 16, 8192)), dim3(256), 0, st, rowptr, col, cnt,
                     D, K, W, P, cd, cpd, invm);
  TSK_TRY(check_launch("k_doc_project"));
  hipLaunchKernelGGL(tsk::k_doc_q_partial<R>, dim3(G), dim3(128), 0, st, (const R*)P, (const double*)invm,
                     D, K, per_q, qpart);
  hipLaunchKernelGGL(tsk::k_doc_q_final, dim3(K + 1), dim3(256), 0, st, (const double*)qpart, G, K, q, deff);
  TSK_TRY(check_launch("k_doc_q"));
  // words: documents containing each word, in document order (stable sort by word)
  int32_t *sdoc = (int32_t*)at(10), *scnt = (int32_t*)at(7);
  TSK_TRY(word_order(rowptr, col, cnt, D, V, nnz, (unsigned long long*)at(7), (unsigned long long*)at(8),
                     (uint32_t*)at(9), at(11), sort_tmp, colptr, sdoc, scnt, st));
  double2* wcd = (double2*)at(24);
  hipLaunchKernelGGL(tsk::k_pack_doc_weights, dim3(grid_for((size_t)D, 256)), dim3(256), 0, st, (const double*)cd,
                     (const double*)cpd, D, wcd);
  TSK_TRY(check_launch("k_pack_doc_weights"));
  hipLaunchKernelGGL(tsk::k_word_accum<R>, dim3(std::min(V, 16384)), dim3(64), 0, st, (const int32_t*)sdoc,
                     (const int32_t*)scnt, (const int32_t*)colptr, (const R*)P, (const double2*)wcd, V, K, Rw, g,
                     gp);
  TSK_TRY(check_launch("k_word_accum"));
  const double a = alpha0 / (alpha0 + 2.0);
  const double c3 = 2.0 * alpha0 * alpha0 / ((alpha0 + 1.0) * (alpha0 + 2.0));
  if (moment) {
    // documents: c_d p^(x)3 and -a c'_d p p^T; words: 2 g w^(x)3, -(w w R) and a g' w w^T
    double* Cd = (double*)at(21);
    double* Cw = (double*)at(22);
    double* T = (double*)at(23);
    TSK_TRY((launch_moment<R, false>(ms, P, nullptr, cd, cpd, 1.0, -a, 0.0, K, D, (double*)at(19), Cd, st)));
    TSK_TRY((launch_moment<R, true>(ms, W, Rw, g, gp, 2.0, a, -1.0, K, V, (double*)at(20), Cw, st)));
    hipLaunchKernelGGL(tsk::k_moment_assemble, dim3(grid_for((size_t)K * K * K, 256)), dim3(256), 0, st,
                       (const double*)Cd, (const double*)Cw, (const double*)q, (const double*)deff, c3, K, T);
    TSK_TRY(check_launch("k_moment_assemble"));
    return tsk_sketch_build_dense(ctx, tab, T, TSK_F64, S64, S32, accumulate, st);
  }
  TSK_TRY(launch_mode_spectra<R>(logb, tab, q, tw, Qs, st));
  tsk::TermArgs ta;
  ta.hxs = tab->hxs;
  ta.ord = tab->ord;
  ta.n = K;
  ta.B = B;
  ta.Qs = Qs;
  ta.twg = tw;
  // documents: c_d p^(x)3 - a c'_d (p p q + p q p + q p p)
  ta.nitem = D;
  ta.per = (D + ncD - 1) / ncD;
  ta.X = P;
  ta.Y = nullptr;
  ta.arrA = cd;
  ta.arrB = cpd;
  ta.sa = 1.0;
  ta.sb = -a;
  ta.gam = 0.0;
  ta.part = partD;
  TSK_TRY((launch_terms<R, false>(logb, ta, B, ncD, st)));
  // words: 2 g w^(x)3 + a g' (w w q + w q w + q w w) - (w w R + w R w + R w w)
  ta.nitem = V;
  ta.per = (V + ncW - 1) / ncW;
  ta.X = W;
  ta.Y = Rw;
  ta.arrA = g;
  ta.arrB = gp;
  ta.sa = 2.0;
  ta.sb = a;
  ta.gam = -1.0;
  ta.part = partW;
  TSK_TRY((launch_terms<R, true>(logb, ta, B, ncW, st)));
  hipLaunchKernelGGL(tsk::k_terms_final<R>, dim3(grid_for((size_t)B * H1, 256)), dim3(256), 0, st,
                     (const cx<double>*)partD, ncD, (const cx<double>*)partW, ncW, (const cx<R>*)Qs,
                     (const double*)deff, c3, B, H1, accumulate, reinterpret_cast<cx<double>*>(S64),
                     reinterpret_cast<cx<float>*>(S32));
  return check_launch("k_terms_final");
}

}  // namespace

extern "C" tsk_status tsk_sketch_build_docs(tsk_ctx_t ctx, tsk_tables_t tab, const int32_t* rowptr,
                                            const int32_t* col, const int32_t* cnt, int D, int V,
                                            const void* W, tsk_dtype wdtype, double alpha0, double* S64,
                                            float* S32, int accumulate, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_sketch_build_docs"));
  if (tab->logb > kLdsLogB)
    return tsk::fail(TSK_EUNSUPPORTED, "tsk_sketch_build_docs: b=%d > 16384 is not built", tab->b);
  if (!rowptr || !W || !S64) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_docs: null argument");
  if (D < 1 || V < 1) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_docs: D=%d, V=%d must be >= 1", D, V);
  if (tab->n > 128)
    return tsk::fail(TSK_EUNSUPPORTED, "tsk_sketch_build_docs: K=%d > 128 columns of the projection", tab->n);
  if (wdtype != TSK_F32 && wdtype != TSK_F64) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_docs: bad dtype");
  if (!(alpha0 >= 0.0) || alpha0 > 1e300)
    return tsk::fail(TSK_EINVAL, "tsk_sketch_build_docs: alpha0=%g must be finite and >= 0", alpha0);
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  int32_t nnz = 0;
  TSK_HIP(hipMemcpyAsync(&nnz, rowptr + D, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TSK_HIP(hipStreamSynchronize(st));
  if (nnz < 0) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_docs: rowptr[D]=%d < 0", nnz);
  if (nnz > 0 && (!col || !cnt)) return tsk::fail(TSK_EINVAL, "tsk_sketch_build_docs: null col or cnt");
  if (wdtype == TSK_F32)
    return build_docs_impl<float>(ctx, tab, rowptr, col, cnt, D, V, nnz, (const float*)W, alpha0, S64, S32,
                                  accumulate, st);
  return build_docs_impl<double>(ctx, tab, rowptr, col, cnt, D, V, nnz, (const double*)W, alpha0, S64,
                                 S32, accumulate, st);
}

// =============================================================================
// Gradients (extensions built on Eq. (3) and Proposition 1)
// =============================================================================

namespace {

// The three mode read-offs of every (vector, sketch) pair into V3[3][L][B][n];
// the mode-1 launch also writes lam_per[L][B] = <s^(m), s^(m)(u^(x)3)>.
template <typename R>
tsk_status three_readoffs(tsk_ctx_t ctx, tsk_tables_t tab, const void* spec, int L, const R* U,
                          R* V3, double* lam_per, hipStream_t st) {
  const size_t blk = (size_t)L * tab->B * tab->n;
  SplitBufs sb;
  TSK_TRY(eager_split_bufs(ctx, tab, sizeof(R) == 4 ? TSK_F32 : TSK_F64, L, &sb));
  for (int perm = 0; perm < 3; ++perm)
    TSK_TRY(power_launch<R>(ctx, tab, spec, L, 0, 0, perm == 0 ? 1 : 0, U, nullptr, nullptr, nullptr,
                            V3 + perm * blk, perm == 0 ? lam_per : nullptr, st, perm, &sb));
  return TSK_OK;
}

}  // namespace

extern "C" tsk_status tsk_contract_tuuu_grad(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype,
                                             const double* S64, const float* S32, int L,
                                             const void* U, const void* scale, double* f_med,
                                             double* f_per, void* grad, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_contract_tuuu_grad"));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, "tsk_contract_tuuu_grad"));
  if (!U || !f_med || !grad) return tsk::fail(TSK_EINVAL, "tsk_contract_tuuu_grad: null U, f_med or grad");
  TSK_TRY(set_device(ctx));
  const size_t es = dtype == TSK_F32 ? 4 : 8;
  const size_t blk = (size_t)L * tab->B * tab->n;
  void* v3 = nullptr;
  TSK_TRY(ws_get(ctx, WS_V3, 3 * blk * es, &v3));
  void* lp = f_per;
  if (!lp) TSK_TRY(ws_get(ctx, WS_LAMPER, (size_t)L * tab->B * sizeof(double), &lp));
  if (dtype == TSK_F32) {
    float* V = (float*)v3;
    TSK_TRY(three_readoffs<float>(ctx, tab, S32, L, (const float*)U, V, (double*)lp, S(stream)));
    hipLaunchKernelGGL(tsk::k_tuuu_grad<float>, dim3(L), dim3(256), 0, S(stream), (const double*)lp, V,
                       V + blk, V + 2 * blk, (const float*)scale, tab->n, tab->B, f_med, (float*)grad);
  } else {
    double* V = (double*)v3;
    TSK_TRY(three_readoffs<double>(ctx, tab, S64, L, (const double*)U, V, (double*)lp, S(stream)));
    hipLaunchKernelGGL(tsk::k_tuuu_grad<double>, dim3(L), dim3(256), 0, S(stream), (const double*)lp, V,
                       V + blk, V + 2 * blk, (const double*)scale, tab->n, tab->B, f_med,
                       (double*)grad);
  }
  return check_launch("k_tuuu_grad");
}

extern "C" tsk_status tsk_cp_loss(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, const double* S64,
                                  int k, const void* lam, const void* U, const void* scale,
                                  double* loss, void* grad_lam, void* grad_U, void* stream) {
  TSK_TRY(check_tables(tab, ctx, "tsk_cp_loss"));
  if (dtype != TSK_F32 && dtype != TSK_F64) return tsk::fail(TSK_EINVAL, "tsk_cp_loss: bad dtype");
  if (!S64 || !lam || !U || !loss) return tsk::fail(TSK_EINVAL, "tsk_cp_loss: null argument");
  if (k < 1 || k > 65535) return tsk::fail(TSK_EINVAL, "tsk_cp_loss: k=%d outside [1, 65535]", k);
  TSK_TRY(set_device(ctx));
  const int B = tab->B, b = tab->b, n = tab->n;
  const size_t H1 = (size_t)b / 2 + 1;
  const hipStream_t st = S(stream);
  void *r64 = nullptr, *r32 = nullptr;
  TSK_TRY(ws_get(ctx, WS_R64, (size_t)B * H1 * sizeof(cx<double>), &r64));
  if (dtype == TSK_F32) TSK_TRY(ws_get(ctx, WS_R32, (size_t)B * H1 * sizeof(cx<float>), &r32));
  TSK_HIP(hipMemcpyAsync(r64, S64, (size_t)B * H1 * sizeof(cx<double>), hipMemcpyDeviceToDevice, st));
  const double* lamd = (const double*)lam;
  const double* Ud = (const double*)U;
  if (dtype == TSK_F32) {
    void *ld = nullptr, *ud = nullptr;
    TSK_TRY(ws_get(ctx, WS_LAMD, (size_t)k * sizeof(double), &ld));
    TSK_TRY(ws_get(ctx, WS_UD, (size_t)k * n * sizeof(double), &ud));
    hipLaunchKernelGGL(tsk::k_widen<float>, dim3(grid_for((size_t)k, 256)), dim3(256), 0, st,
                       (const float*)lam, (double*)ld, (size_t)k);
    hipLaunchKernelGGL(tsk::k_widen<float>, dim3(grid_for((size_t)k * n, 256)), dim3(256), 0, st,
                       (const float*)U, (double*)ud, (size_t)k * n);
    TSK_TRY(check_launch("k_widen"));
    lamd = (const double*)ld;
    Ud = (const double*)ud;
  }
  // residual spectra R = S - sum_i lam_i prod_j F(s_j u_i), FP64 (and FP32 copy)
  TSK_TRY(rank1_update(ctx, tab, lamd, Ud, k, -1.0, (double*)r64, (float*)r32, st));
  hipLaunchKernelGGL(tsk::k_parseval_loss, dim3(1), dim3(1024), 0, st, (const cx<double>*)r64, B, b, loss);
  TSK_TRY(check_launch("k_parseval_loss"));
  if (!grad_lam && !grad_U) return TSK_OK;
  const size_t es = dtype == TSK_F32 ? 4 : 8;
  const size_t blk = (size_t)k * B * n;
  void *v3 = nullptr, *lp = nullptr;
  TSK_TRY(ws_get(ctx, WS_V3, 3 * blk * es, &v3));
  TSK_TRY(ws_get(ctx, WS_LAMPER, (size_t)k * B * sizeof(double), &lp));
  if (dtype == TSK_F32) {
    float* V = (float*)v3;
    TSK_TRY(three_readoffs<float>(ctx, tab, r32, k, (const float*)U, V, (double*)lp, st));
    hipLaunchKernelGGL(tsk::k_cp_grad<float>, dim3(k), dim3(256), 0, st, (const double*)lp, V, V + blk,
                       V + 2 * blk, (const float*)lam, (const float*)scale, n, B, (float*)grad_lam,
                       (float*)grad_U);
  } else {
    double* V = (double*)v3;
    TSK_TRY(three_readoffs<double>(ctx, tab, r64, k, (const double*)U, V, (double*)lp, st));
    hipLaunchKernelGGL(tsk::k_cp_grad<double>, dim3(k), dim3(256), 0, st, (const double*)lp, V, V + blk,
                       V + 2 * blk, (const double*)lam, (const double*)scale, n, B, (double*)grad_lam,
                       (double*)grad_U);
  }
  return check_launch("k_cp_grad");
}

// =============================================================================
// Decomposition
// =============================================================================

namespace {

struct DecompWs {
  void* U0r;      // R[k][L][n] the start vectors in the power steps' precision
  void* U0;       // R[L][n]
  void* U1;       // R[L][n]
  void* V0;       // R[L][B][n]
  void* V1;       // R[L][B][n]
  double* lam_per;
  double* lam_med;
  int32_t* flags;  // [k][L]
  double* u_hat;   // [n]
  double* lam64;   // [B]
  void* prod;      // cx<double>[B][b/2+1]
  double* u0;      // [k][L][n] generated start vectors (when caller passes none)
  void* esplit;    // split rank-1 sub-transforms (b >= 16384)
  SplitBufs sb;    // split FP32 power steps (b = 65536)
};

// Power steps of one component for restarts [tau0, tau0 + nrest): the first
// step uses u0 directly, every later launch (and the final evaluation) starts
// from the normalised median of the previous launch's estimates.  Returns the
// buffer holding u_T.
template <typename R>
tsk_status power_chain(tsk_ctx_t ctx, tsk_tables_t tab, const void* spec, int nrest, int tau0, int T,
                       const R* u_start, R* const Ub[2], R* const Vb[2], double* lam_per, int32_t* fl,
                       R** u_final, hipStream_t st, const SplitBufs* sb) {
  TSK_TRY(power_launch<R>(ctx, tab, spec, nrest, tau0, 0, 0, u_start, nullptr, nullptr, nullptr, Vb[0],
                          nullptr, st, 0, sb));
  const R* uprev = u_start;  // the fallback of a step whose median is unusable
  for (int t = 1; t <= T; ++t) {
    const int mode = (t == T) ? 1 : 0;
    R* ucur = Ub[t & 1];
    TSK_TRY(power_launch<R>(ctx, tab, spec, nrest, tau0, 1, mode, uprev, Vb[(t - 1) & 1], ucur, fl,
                            Vb[t & 1], mode ? lam_per : nullptr, st, 0, sb));
    uprev = ucur;
  }
  *u_final = Ub[T & 1];
  return TSK_OK;
}

template <typename R>
tsk_status decompose_enqueue(tsk_ctx_t ctx, tsk_tables_t tab, const void* spec, double* S64,
                             float* S32, int k, int L, int T, const double* u0, double* lam_out,
                             double* U_out, int32_t* tau_out, int32_t* flags, const DecompWs& w,
                             bool plain, int groups, hipStream_t st) {
  const int n = tab->n, B = tab->B, b = tab->b;
  const int H1 = b / 2 + 1;
  const cx<double>* tw64 = nullptr;
  if (tab->logb <= kLdsLogB) TSK_TRY(get_tw<double>(ctx, tab->logb, &tw64));
  R* const Ub[2] = {reinterpret_cast<R*>(w.U0), reinterpret_cast<R*>(w.U1)};
  R* const Vb[2] = {reinterpret_cast<R*>(w.V0), reinterpret_cast<R*>(w.V1)};
  // The start vectors of every component in the power steps' precision, in
  // one launch ahead of the component loop (off the chain of dependent steps).
  const size_t LN = (size_t)L * n;
  R* const U0r = reinterpret_cast<R*>(w.U0r);
  hipLaunchKernelGGL(tsk::k_cvt<R>, dim3(grid_for((size_t)k * LN, 256)), dim3(256), 0, st, u0, U0r,
                     (size_t)k * LN);
  TSK_TRY(check_launch("k_cvt"));
  for (int c = 0; c < k; ++c) {
    const R* us = U0r + (size_t)c * LN;
    int32_t* fl = flags + (size_t)c * L;
    R* ufin = nullptr;
    if (!plain && groups > 1) {
      // The restarts are independent until the selection: G groups of them
      // run their T + 1 steps on parallel branches, so one group's launch
      // tail overlaps the others' work.
      TSK_HIP(hipEventRecord(ctx->gfork_ev[groups], st));
      for (int g = 0; g < groups; ++g) {
        const int t0 = (int)((long)L * g / groups), t1 = (int)((long)L * (g + 1) / groups);
        hipStream_t s = ctx->gfork[g];
        TSK_HIP(hipStreamWaitEvent(s, ctx->gfork_ev[groups], 0));
        TSK_TRY(power_chain<R>(ctx, tab, spec, t1 - t0, t0, T, us, Ub, Vb, w.lam_per, fl, &ufin, s, &w.sb));
        TSK_HIP(hipEventRecord(ctx->gfork_ev[g], s));
        TSK_HIP(hipStreamWaitEvent(st, ctx->gfork_ev[g], 0));
      }
    } else if (!plain) {
      TSK_TRY(power_chain<R>(ctx, tab, spec, L, 0, T, us, Ub, Vb, w.lam_per, fl, &ufin, st, &w.sb));
    } else {
      for (int tau = 0; tau < L; ++tau)
        TSK_TRY(power_chain<R>(ctx, tab, spec, 1, tau, T, us, Ub, Vb, w.lam_per, fl, &ufin, st, &w.sb));
    }
    TSK_TRY(lam_median_launch(w.lam_per, w.lam_med, L, B, st));
    hipLaunchKernelGGL(tsk::k_select<R>, dim3(1), dim3(256), 0, st, (const double*)w.lam_med, L,
                       (const R*)ufin, n, w.u_hat, U_out + (size_t)c * n,
                       tau_out ? tau_out + c : nullptr);
    TSK_TRY(check_launch("k_select"));
    tsk::Rank1Args a;
    a.hx = tab->hx;
    a.hxs = tab->hxs;
    a.ord = tab->ord;
    a.n = n;
    a.B = B;
    a.U = w.u_hat;
    a.twg = tw64;
    a.prod = reinterpret_cast<cx<double>*>(w.prod);
    a.S64 = reinterpret_cast<const cx<double>*>(S64);
    a.lam_per = w.lam64;
    TSK_TRY(launch_rank1_any(ctx, tab, a, 1, w.esplit, st));
    hipLaunchKernelGGL(tsk::k_spec_deflate, dim3(grid_for((size_t)B * H1, 256)), dim3(256), 0, st,
                       reinterpret_cast<cx<double>*>(S64), reinterpret_cast<cx<float>*>(S32),
                       (const cx<double>*)w.prod, (const double*)w.lam64, B, H1, lam_out + c);
    TSK_TRY(check_launch("k_spec_deflate"));
  }
  return TSK_OK;
}

}  // namespace

namespace {

tsk_status check_decompose(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, const double* S64,
                           const float* S32, int k, int L, int T, const double* u0,
                           const double* lam_out, const double* U_out, const char* fn) {
  TSK_TRY(check_tables(tab, ctx, fn));
  TSK_TRY(check_power_args(tab, dtype, S64, S32, L, fn));
  if (!S64) return tsk::fail(TSK_EINVAL, "%s: S64 (deflated in FP64) is required", fn);
  if (!lam_out || !U_out) return tsk::fail(TSK_EINVAL, "%s: null lam_out or U_out", fn);
  if (k < 1 || k > tab->n) return tsk::fail(TSK_EINVAL, "%s: k=%d outside [1,n]", fn, k);
  if (T < 1) return tsk::fail(TSK_EINVAL, "%s: T=%d < 1", fn, T);
  if (!u0 && (L >= (1 << 20) || tab->n >= (1 << 19)))
    return tsk::fail(TSK_EINVAL, "%s: too large to draw start vectors", fn);
  return TSK_OK;
}

// Workspace of one decomposition carved from one buffer (256-byte aligned
// pieces); with base == nullptr only the size is computed.
size_t decomp_ws_layout(char* base, tsk_tables_t tab, tsk_dtype dtype, int k, int L, bool flags,
                        bool u0, DecompWs* w, int32_t** fl, double** u0p) {
  const size_t n = tab->n, B = tab->B, H1 = (size_t)tab->b / 2 + 1;
  const size_t es = dtype == TSK_F32 ? 4 : 8;
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  DecompWs d;
  d.U0r = take((size_t)k * L * n * es);
  d.U0 = take(L * n * es);
  d.U1 = take(L * n * es);
  d.V0 = take(L * B * n * es);
  d.V1 = take(L * B * n * es);
  d.lam_per = (double*)take(L * B * 8);
  d.lam_med = (double*)take((size_t)L * 8);
  d.u_hat = (double*)take(n * 8);
  d.lam64 = (double*)take(B * 8);
  d.prod = take(B * H1 * 16);
  d.flags = flags ? (int32_t*)take((size_t)k * L * 4) : nullptr;
  d.u0 = u0 ? (double*)take((size_t)k * L * n * 8) : nullptr;
  d.esplit = rank1_split_path(tab->logb) ? take(rank1_split_bytes(tab, 1)) : nullptr;
  if (needs_power_split(tab, dtype)) {
    d.sb.A = take(power_split_bytes_A(tab, L));
  }
  if (w) *w = d;
  if (fl) *fl = d.flags;
  if (u0p) *u0p = d.u0;
  return off;
}

tsk_status upload_start_vectors(uint64_t seed, int k, int L, int n, double* dst, hipStream_t st) {
  std::vector<double> h((size_t)k * L * n);
  for (int c = 0; c < k; ++c) TSK_TRY(tsk_init_vectors(seed, c, L, n, h.data() + (size_t)c * L * n));
  TSK_HIP(hipStreamSynchronize(st));
  TSK_HIP(hipMemcpy(dst, h.data(), h.size() * 8, hipMemcpyHostToDevice));
  return TSK_OK;
}

tsk_status preload_twiddles(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype) {
  const cx<double>* t64 = nullptr;
  const cx<float>* t32 = nullptr;
  if (tab->logb <= kLdsLogB) TSK_TRY(get_tw<double>(ctx, tab->logb, &t64));
  if (dtype == TSK_F32 && tab->logb <= kLdsLogB + 1) TSK_TRY(get_tw<float>(ctx, tab->logb, &t32));
  return preload_split_tables(ctx, tab->logb, needs_power_split(tab, dtype));
}

// Streams for `count` graph branches and count + 1 events (the last one forks).
tsk_status ensure_branches(std::vector<hipStream_t>& streams, std::vector<hipEvent_t>& events, int count) {
  while ((int)streams.size() < count) {
    hipStream_t s = nullptr;
    TSK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    streams.push_back(s);
  }
  while ((int)events.size() < count + 1) {
    hipEvent_t e = nullptr;
    TSK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    events.push_back(e);
  }
  return TSK_OK;
}

// Parallel restart groups of one decomposition.  Two halves of the restarts
// on two branches measured fastest (their launches overlap each other's
// start-up and tail; three or four branches gained less).  The split power
// step (one work-group per CU) takes two groups only when one launch would
// need more than one round of the 256 CUs (B = 16, L = 30: 22.9 -> 21.3 ms per
// decomposition; B = 8, L = 30: 8.3 -> 8.5 ms with two); its scratch rows are
// indexed by restart, so the groups share nothing.
int restart_groups(tsk_tables_t tab, tsk_dtype dtype, int L) {
  if (L < 2) return 1;
  if (needs_power_split(tab, dtype)) return (long)tab->B * L > 256 ? 2 : 1;
  return 2;
}

// Everything one decomposition enqueues: clear its flags (a fill kernel, so a
// recorded graph holds no memset node), then the component loop.
tsk_status decompose_all(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, double* S64, float* S32,
                         int k, int L, int T, const double* u0d, double* lam_out, double* U_out,
                         int32_t* tau_out, int32_t* flags, const DecompWs& w, bool plain,
                         int groups, hipStream_t s) {
  hipLaunchKernelGGL(tsk::k_fill_u32, dim3(grid_for((size_t)k * L, 256)), dim3(256), 0, s,
                     reinterpret_cast<unsigned*>(flags), 0u, (size_t)k * L);
  TSK_TRY(check_launch("k_fill_u32"));
  const void* spec = dtype == TSK_F32 ? (const void*)S32 : (const void*)S64;
  if (dtype == TSK_F32)
    return decompose_enqueue<float>(ctx, tab, spec, S64, S32, k, L, T, u0d, lam_out, U_out, tau_out,
                                    flags, w, plain, groups, s);
  return decompose_enqueue<double>(ctx, tab, spec, S64, S32, k, L, T, u0d, lam_out, U_out, tau_out,
                                   flags, w, plain, groups, s);
}

GraphEntry* find_graph(tsk_ctx_t ctx, const std::vector<uint64_t>& key) {
  for (auto& g : ctx->graphs)
    if (g.key == key) return &g;
  return nullptr;
}

// Record what `enqueue(stream)` launches on the capture stream into a graph
// and keep it under `key`.
template <typename F>
tsk_status record_graph(tsk_ctx_t ctx, const std::vector<uint64_t>& key, F enqueue, GraphEntry** out) {
  GraphEntry g;
  g.key = key;
  TSK_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed));
  tsk_status s = enqueue(ctx->cap);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
  if (s != TSK_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return tsk::fail(TSK_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  g.graph = graph;
  TSK_HIP(hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
  if (ctx->graphs.size() >= 16) clear_graphs(ctx);
  ctx->graphs.push_back(g);
  *out = &ctx->graphs.back();
  return TSK_OK;
}

}  // namespace

extern "C" tsk_status tsk_decompose(tsk_ctx_t ctx, tsk_tables_t tab, tsk_dtype dtype, double* S64,
                                    float* S32, int k, int L, int T, const double* u0,
                                    uint64_t seed, double* lam_out, double* U_out,
                                    int32_t* tau_out, int32_t* flags_out, int plain,
                                    void* stream) {
  TSK_TRY(check_decompose(ctx, tab, dtype, S64, S32, k, L, T, u0, lam_out, U_out, "tsk_decompose"));
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  const int n = tab->n;
  int groups = ctx->force_groups > 0 ? std::min(ctx->force_groups, L) : restart_groups(tab, dtype, L);
  if (!plain && ctx->force_groups == 0 && ctx->tune_mode != 0 && L >= 2) {
    // Restart groups: each candidate times a one-component decomposition of
    // the same sizes on a copy of the sketch (the choice does not change the
    // arithmetic of any restart).
    const std::string key = tune_key(ctx, "decompose", dtype, {n, tab->b, tab->B, L, T});
    std::vector<int> cands = {groups};  // the rule first
    for (int g = 1; g <= std::min(4, L); ++g)
      if (g != groups) cands.push_back(g);
    const size_t H1 = (size_t)tab->b / 2 + 1;
    const size_t b64 = ((size_t)tab->B * H1 * 16 + 255) & ~(size_t)255;
    const size_t b32 = ((size_t)tab->B * H1 * 8 + 255) & ~(size_t)255;
    auto time_one = [&](const int& g, float* ms) -> tsk_status {
      void* tb = nullptr;
      TSK_TRY(ws_get(ctx, WS_TUNE, b64 + b32 + 8 + (size_t)n * 8 + 256, &tb));
      double* s64 = (double*)tb;
      float* s32 = (float*)((char*)tb + b64);
      double* lam1 = (double*)((char*)tb + b64 + b32);
      double* u1 = lam1 + 1;
      TSK_HIP(hipMemcpyAsync(s64, S64, (size_t)tab->B * H1 * 16, hipMemcpyDeviceToDevice, st));
      if (S32) TSK_HIP(hipMemcpyAsync(s32, S32, (size_t)tab->B * H1 * 8, hipMemcpyDeviceToDevice, st));
      ctx->force_groups = g;
      const tsk_status s = time_runs(st, 2, [&]() {
        return tsk_decompose(ctx, tab, dtype, s64, s32, 1, L, T, nullptr, 0, lam1, u1, nullptr, nullptr, 0,
                             stream);
      }, ms);
      ctx->force_groups = 0;
      return s;
    };
    auto encode = [](const int& g) { return std::vector<int>{g}; };
    const std::vector<int>* ch = nullptr;
    TSK_TRY(tune_choose(ctx, key, cands, +encode, time_one, &ch));
    if (ch && !ch->empty()) groups = std::max(1, std::min((*ch)[0], L));
  }
  const size_t bytes = decomp_ws_layout(nullptr, tab, dtype, k, L, !flags_out, false, nullptr, nullptr,
                                        nullptr);
  // Generated start vectors live in a slot of their own: other entry points
  // (the symmetric decomposition) lay their scratch over WS_U.
  double* u0_ws = nullptr;
  if (!u0) TSK_TRY(ws_get(ctx, WS_U0, (size_t)k * L * n * 8, (void**)&u0_ws));
  void* base = nullptr;
  TSK_TRY(ws_get(ctx, WS_U, bytes, &base));
  DecompWs w;
  int32_t* fl_ws = nullptr;
  decomp_ws_layout((char*)base, tab, dtype, k, L, !flags_out, false, &w, &fl_ws, nullptr);
  int32_t* flags = flags_out ? flags_out : fl_ws;
  const double* u0d = u0;
  if (!u0d) {
    std::vector<uint64_t> key = {seed, (uint64_t)k, (uint64_t)L, (uint64_t)n, (uint64_t)(uintptr_t)u0_ws};
    if (ctx->u0_key != key) {
      TSK_TRY(upload_start_vectors(seed, k, L, n, u0_ws, st));
      ctx->u0_key = key;
    }
    u0d = u0_ws;
  }
  TSK_TRY(preload_twiddles(ctx, tab, dtype));  // uploads stay outside any capture
  if (!plain) TSK_TRY(ensure_branches(ctx->gfork, ctx->gfork_ev, groups));
  auto enqueue = [&](hipStream_t s) -> tsk_status {
    return decompose_all(ctx, tab, dtype, S64, S32, k, L, T, u0d, lam_out, U_out, tau_out, flags, w,
                         plain != 0, groups, s);
  };
  if (plain) return enqueue(st);
  std::vector<uint64_t> key = {0, (uint64_t)(uintptr_t)tab, (uint64_t)dtype, (uint64_t)(uintptr_t)S64,
                               (uint64_t)(uintptr_t)S32, (uint64_t)k, (uint64_t)L, (uint64_t)T,
                               (uint64_t)(uintptr_t)u0d, (uint64_t)(uintptr_t)lam_out,
                               (uint64_t)(uintptr_t)U_out, (uint64_t)(uintptr_t)tau_out,
                               (uint64_t)(uintptr_t)flags, (uint64_t)(uintptr_t)base, (uint64_t)groups};
  GraphEntry* ge = find_graph(ctx, key);
  if (!ge) TSK_TRY(record_graph(ctx, key, enqueue, &ge));
  TSK_HIP(hipGraphLaunch(ge->exec, st));
  return TSK_OK;
}

extern "C" tsk_status tsk_decompose_batched(tsk_ctx_t ctx, int ninst, const tsk_problem* probs,
                                            void* stream) {
  if (!ctx || !probs) return tsk::fail(TSK_EINVAL, "tsk_decompose_batched: null argument");
  if (ninst < 1) return tsk::fail(TSK_EINVAL, "tsk_decompose_batched: ninst=%d < 1", ninst);
  for (int i = 0; i < ninst; ++i) {
    const tsk_problem& p = probs[i];
    tsk_status s = check_decompose(ctx, p.tab, p.dtype, p.S64, p.S32, p.k, p.L, p.T, p.u0, p.lam_out,
                                   p.U_out, "tsk_decompose_batched");
    if (s != TSK_OK) {
      const std::string msg = tsk_last_error();
      return tsk::fail(s, "tsk_decompose_batched: instance %d: %s", i, msg.c_str());
    }
  }
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  // one workspace buffer, instances at fixed offsets
  std::vector<size_t> off(ninst);
  size_t total = 0;
  for (int i = 0; i < ninst; ++i) {
    const tsk_problem& p = probs[i];
    off[i] = total;
    total += decomp_ws_layout(nullptr, p.tab, p.dtype, p.k, p.L, !p.flags_out, !p.u0, nullptr, nullptr,
                              nullptr);
  }
  void* base = nullptr;
  TSK_TRY(ws_get(ctx, WS_BATCH, total, &base));
  std::vector<DecompWs> w(ninst);
  std::vector<int32_t*> flags(ninst);
  std::vector<const double*> u0d(ninst);
  std::vector<uint64_t> u0key = {(uint64_t)(uintptr_t)base};
  for (int i = 0; i < ninst; ++i) {
    const tsk_problem& p = probs[i];
    int32_t* fl = nullptr;
    double* u0w = nullptr;
    decomp_ws_layout((char*)base + off[i], p.tab, p.dtype, p.k, p.L, !p.flags_out, !p.u0, &w[i], &fl,
                     &u0w);
    flags[i] = p.flags_out ? p.flags_out : fl;
    u0d[i] = p.u0 ? p.u0 : u0w;
    if (!p.u0) {
      u0key.push_back(i);
      u0key.push_back(p.seed);
      u0key.push_back(((uint64_t)p.k << 40) | ((uint64_t)p.L << 20) | (uint64_t)p.tab->n);
      u0key.push_back(off[i]);
    }
    TSK_TRY(preload_twiddles(ctx, p.tab, p.dtype));
  }
  if (ctx->u0b_key != u0key) {
    for (int i = 0; i < ninst; ++i)
      if (!probs[i].u0)
        TSK_TRY(upload_start_vectors(probs[i].seed, probs[i].k, probs[i].L, probs[i].tab->n,
                                     const_cast<double*>(u0d[i]), st));
    ctx->u0b_key = u0key;
  }
  // Longest-first assignment of instances to at most 32 graph branches by
  // their sketch-update work k L (T+1) B b log2 b.  More branches keep more
  // of the small instances' launches in flight beside the large ones (64
  // uneven instances: 4, 8, 16, 32, 64 branches took 2.20, 1.94, 1.76, 1.70,
  // 1.69 s).
  const int nb = std::min(ninst, 32);
  TSK_TRY(ensure_branches(ctx->fork, ctx->fork_ev, nb));
  std::vector<int> order(ninst);
  std::vector<double> work(ninst);
  for (int i = 0; i < ninst; ++i) {
    const tsk_problem& p = probs[i];
    order[i] = i;
    work[i] = (double)p.k * p.L * (p.T + 1) * p.tab->B * (double)p.tab->b * p.tab->logb;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
  std::vector<std::vector<int>> branch(nb);
  std::vector<double> load(nb, 0.0);
  for (int i : order) {
    const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    branch[j].push_back(i);
    load[j] += work[i];
  }
  std::vector<uint64_t> key = {1, (uint64_t)ninst, (uint64_t)(uintptr_t)base};
  for (int i = 0; i < ninst; ++i) {
    const tsk_problem& p = probs[i];
    const uint64_t v[] = {(uint64_t)(uintptr_t)p.tab, (uint64_t)p.dtype, (uint64_t)(uintptr_t)p.S64,
                          (uint64_t)(uintptr_t)p.S32, (uint64_t)p.k, (uint64_t)p.L, (uint64_t)p.T,
                          (uint64_t)(uintptr_t)u0d[i], (uint64_t)(uintptr_t)p.lam_out,
                          (uint64_t)(uintptr_t)p.U_out, (uint64_t)(uintptr_t)p.tau_out,
                          (uint64_t)(uintptr_t)flags[i]};
    key.insert(key.end(), std::begin(v), std::end(v));
  }
  auto enqueue = [&](hipStream_t cap) -> tsk_status {
    TSK_HIP(hipEventRecord(ctx->fork_ev[nb], cap));
    for (int j = 0; j < nb; ++j) {
      hipStream_t s = ctx->fork[j];
      TSK_HIP(hipStreamWaitEvent(s, ctx->fork_ev[nb], 0));
      for (int i : branch[j]) {
        const tsk_problem& p = probs[i];
        TSK_TRY(decompose_all(ctx, p.tab, p.dtype, p.S64, p.S32, p.k, p.L, p.T, u0d[i], p.lam_out,
                              p.U_out, p.tau_out, flags[i], w[i], false, 1, s));
      }
      TSK_HIP(hipEventRecord(ctx->fork_ev[j], s));
      TSK_HIP(hipStreamWaitEvent(cap, ctx->fork_ev[j], 0));
    }
    return TSK_OK;
  };
  GraphEntry* ge = find_graph(ctx, key);
  if (!ge) TSK_TRY(record_graph(ctx, key, enqueue, &ge));
  TSK_HIP(hipGraphLaunch(ge->exec, st));
  return TSK_OK;
}

extern "C" tsk_status tsk_workspace_size(tsk_ctx_t ctx, int ninst, const tsk_problem* probs,
                                         size_t* bytes) {
  if (!ctx || !probs || !bytes) return tsk::fail(TSK_EINVAL, "tsk_workspace_size: null argument");
  if (ninst < 1) return tsk::fail(TSK_EINVAL, "tsk_workspace_size: ninst=%d < 1", ninst);
  size_t total = 0;
  for (int i = 0; i < ninst; ++i) {
    const tsk_problem& p = probs[i];
    TSK_TRY(check_decompose(ctx, p.tab, p.dtype, p.S64, p.S32, p.k, p.L, p.T, p.u0, p.lam_out, p.U_out,
                            "tsk_workspace_size"));
    total += decomp_ws_layout(nullptr, p.tab, p.dtype, p.k, p.L, !p.flags_out, !p.u0, nullptr, nullptr,
                              nullptr);
  }
  *bytes = total;
  return TSK_OK;
}

// =============================================================================
// Colliding-hash symmetric sketches (Section 3.3, Appendix B)
// =============================================================================

extern "C" tsk_status tsk_sym_tables_create(tsk_ctx_t ctx, int n, int b, int B, const uint32_t* h_host,
                                            const uint8_t* q_host, tsk_sym_tables_t* out) {
  if (!ctx || !h_host || !q_host || !out) return tsk::fail(TSK_EINVAL, "tsk_sym_tables_create: null argument");
  if (n < 1 || n > 65535 || B < 1 || B > 64)
    return tsk::fail(TSK_EINVAL, "tsk_sym_tables_create: n=%d, B=%d out of range", n, B);
  if (b < 256 || b > 65536 || (b & (b - 1)))
    return tsk::fail(TSK_EUNSUPPORTED, "tsk_sym_tables_create: b=%d (powers of two in [256, 65536])", b);
  const size_t cnt = (size_t)B * n;
  std::vector<uint32_t> hq(cnt), srt(3 * cnt), ord(3 * cnt);
  for (size_t e = 0; e < cnt; ++e) {
    if (h_host[e] >= (uint32_t)b || q_host[e] > 3)
      return tsk::fail(TSK_EINVAL, "tsk_sym_tables_create: h or q out of range at %zu", e);
    hq[e] = (h_host[e] << 2) | q_host[e];
  }
  std::vector<uint32_t> idx(n);
  for (int p = 1; p <= 3; ++p)
    for (int m = 0; m < B; ++m) {
      const size_t base = (size_t)m * n, ob = ((size_t)(p - 1) * B + m) * n;
      auto pos = [&](uint32_t i) { return (uint32_t)(((uint64_t)p * h_host[base + i]) & (uint32_t)(b - 1)); };
      std::iota(idx.begin(), idx.end(), 0u);
      std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) { return pos(x) < pos(y); });
      for (int r = 0; r < n; ++r) {
        const uint32_t i = idx[r];
        srt[ob + r] = (pos(i) << 2) | ((uint32_t)(p * q_host[base + i]) & 3u);
        ord[ob + r] = i;
      }
    }
  TSK_TRY(set_device(ctx));
  tsk_sym_tables* t = new tsk_sym_tables;
  t->ctx = ctx;
  t->n = n;
  t->b = b;
  t->B = B;
  t->logb = 0;
  while ((1 << t->logb) < b) ++t->logb;
  if (hipMalloc(&t->hq, 7 * cnt * 4) != hipSuccess) {
    delete t;
    return tsk::fail(TSK_ENOMEM, "tsk_sym_tables_create: device allocation");
  }
  t->srt = t->hq + cnt;
  t->ord = t->srt + 3 * cnt;
  hipError_t e1 = hipMemcpy(t->hq, hq.data(), cnt * 4, hipMemcpyHostToDevice);
  hipError_t e2 = hipMemcpy(t->srt, srt.data(), 3 * cnt * 4, hipMemcpyHostToDevice);
  hipError_t e3 = hipMemcpy(t->ord, ord.data(), 3 * cnt * 4, hipMemcpyHostToDevice);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
    (void)hipFree(t->hq);
    delete t;
    return tsk::fail(TSK_EHIP, "tsk_sym_tables_create: upload failed");
  }
  *out = t;
  return TSK_OK;
}

extern "C" void tsk_sym_tables_destroy(tsk_sym_tables_t t) {
  if (!t) return;
  (void)hipSetDevice(t->ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(t->hq);
  if (t->ef) (void)hipFree(t->ef);
  delete t;
}

namespace {

tsk_status check_sym(tsk_sym_tables_t tab, tsk_ctx_t ctx, const char* fn) {
  if (!ctx) return tsk::fail(TSK_EINVAL, "%s: null context", fn);
  if (!tab) return tsk::fail(TSK_EINVAL, "%s: null tables", fn);
  if (tab->ctx != ctx) return tsk::fail(TSK_EINVAL, "%s: tables belong to another context", fn);
  return TSK_OK;
}

template <int LOGN, bool INV, int DEC>
tsk_status launch_c2c64_t(tsk_ctx_t ctx, const cx<double>* in, cx<double>* out, int rows, hipStream_t st) {
  constexpr int NT = tsk::threads_for_h<double>(LOGN);
  const cx<double>* tw = nullptr;
  TSK_TRY(get_tw<double>(ctx, LOGN + 1, &tw, NT));
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  const size_t lds = sizeof(double) * 2 * (size_t)tsk::padded_len(1 << LOGN);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_c2c64<LOGN, INV, DEC>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL((tsk::k_c2c64<LOGN, INV, DEC>), dim3(rows), dim3(NT), lds, st, in, out, tw);
  return check_launch("k_c2c64");
}

// Complex FFT (unnormalised; inverse with conjugate twiddles) of `rows` rows
// of b = 2^logb points, FP64, with an optional FP32 copy of the result:
// one work-group per row up to 8192 points; above, R = b / 8192 transforms of
// the residue classes mod R per row and a radix-R combination.
tsk_status fft64_rows(tsk_ctx_t ctx, int logb, const cx<double>* in, cx<double>* out, cx<float>* out32, int rows,
                      bool inv, hipStream_t st) {
  const size_t count = (size_t)rows << logb;
  if (logb >= 14 && logb <= 16) {
    const int R = 1 << (logb - 13);
    void* half = nullptr;
    TSK_TRY(ws_get(ctx, WS_SYM, count * sizeof(cx<double>), &half));
    const cx<double>* wb = nullptr;
    TSK_TRY(get_wb<double>(ctx, logb, &wb));
    cx<double>* hb = reinterpret_cast<cx<double>*>(half);
    if (R == 2) {
      if (inv) TSK_TRY((launch_c2c64_t<13, true, 2>(ctx, in, hb, R * rows, st)));
      else TSK_TRY((launch_c2c64_t<13, false, 2>(ctx, in, hb, R * rows, st)));
    } else if (R == 4) {
      if (inv) TSK_TRY((launch_c2c64_t<13, true, 4>(ctx, in, hb, R * rows, st)));
      else TSK_TRY((launch_c2c64_t<13, false, 4>(ctx, in, hb, R * rows, st)));
    } else {
      if (inv) TSK_TRY((launch_c2c64_t<13, true, 8>(ctx, in, hb, R * rows, st)));
      else TSK_TRY((launch_c2c64_t<13, false, 8>(ctx, in, hb, R * rows, st)));
    }
    hipLaunchKernelGGL(tsk::k_c2c_combine, dim3(grid_for(count, 256)), dim3(256), 0, st, (const cx<double>*)hb,
                       out, out32, wb, 1 << 13, R, rows, inv ? 1 : 0);
    return check_launch("k_c2c_combine");
  }
#define TSK_C2C(L)                                                                                      \
  case L:                                                                                               \
    if (inv) TSK_TRY((launch_c2c64_t<L, true, 1>(ctx, in, out, rows, st)));                            \
    else TSK_TRY((launch_c2c64_t<L, false, 1>(ctx, in, out, rows, st)));                               \
    break;
  switch (logb) {
    TSK_C2C(8)
    TSK_C2C(9)
    TSK_C2C(10)
    TSK_C2C(11)
    TSK_C2C(12)
    TSK_C2C(13)
    default: return tsk::fail(TSK_EUNSUPPORTED, "symmetric sketches: b=2^%d", logb);
  }
#undef TSK_C2C
  if (out32) {
    hipLaunchKernelGGL(tsk::k_c64to32, dim3(grid_for(count, 256)), dim3(256), 0, st, (const cx<double>*)out,
                       out32, count);
    TSK_TRY(check_launch("k_c64to32"));
  }
  return TSK_OK;
}

template <int LOGB>
tsk_status launch_sym_power_t(const tsk::SymPowerArgs& a, int L, hipStream_t st) {
  constexpr int NT = tsk::sym_threads(LOGB);
  const size_t lds = tsk::sym_power_lds(LOGB, a.n);
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_sym_power<LOGB>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLds - 256)));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL((tsk::k_sym_power<LOGB>), dim3(a.B, L), dim3(NT), lds, st, a);
  return check_launch("k_sym_power");
}

template <typename K>
tsk_status allow_lds(K* kernel, size_t bytes) {
  (void)bytes;
  TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(kMaxLds - 256)));
  return TSK_OK;
}

// The symmetric step at b = R 16384 through the split transforms (three
// launches, buffer E of L B (R + R/2) rows of 16384 complex values).
template <int R>
tsk_status sym_power_split_t(tsk_ctx_t ctx, tsk_sym_tables_t tab, const float* S32, const float* s32, int L,
                             const float* U, float* V, double* lam_per, int mode, hipStream_t st) {
  constexpr int M = 1 << tsk::kSymSplitLogM, NR = R + R / 2;
  constexpr int NT = tsk::sym_threads(tsk::kSymSplitLogM);
  const size_t lds = tsk::sym_split_lds(tab->n);
  if (lds > kMaxLds - 256)
    return tsk::fail(TSK_EUNSUPPORTED, "symmetric power step: n=%d too large for b=%d", tab->n, tab->b);
  const cx<float>* twM = nullptr;
  const cx<float>* Wb = nullptr;
  TSK_TRY(get_tw<float>(ctx, tsk::kSymSplitLogM + 1, &twM, NT));
  TSK_TRY(get_wb<float>(ctx, tab->logb, &Wb));
  void* E = nullptr;
  TSK_TRY(ws_get(ctx, WS_SYMSPLIT, (size_t)L * tab->B * NR * M * sizeof(cx<float>), &E));
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_TRY(allow_lds(&tsk::k_sym_split_fwd<R>, lds));
    TSK_TRY(allow_lds(&tsk::k_sym_split_out<R>, lds));
    configured.fetch_or(bit);
  }
  tsk::SymSplitArgs a;
  const size_t cnt = (size_t)tab->B * tab->n;
  a.hq = tab->hq;
  a.srt1 = tab->srt;
  a.ord1 = tab->ord;
  a.srt2 = tab->srt + cnt;
  a.ord2 = tab->ord + cnt;
  a.n = tab->n;
  a.B = tab->B;
  a.b = tab->b;
  a.S = reinterpret_cast<const cx<float>*>(S32);
  a.s = reinterpret_cast<const cx<float>*>(s32);
  a.twM = twM;
  a.Wb = Wb;
  a.U = U;
  a.E = reinterpret_cast<cx<float>*>(E);
  a.V = V;
  a.lam_per = lam_per;
  a.mode = mode;
  hipLaunchKernelGGL((tsk::k_sym_split_fwd<R>), dim3(tab->B, L, NR), dim3(NT), lds, st, a);
  TSK_TRY(check_launch("k_sym_split_fwd"));
  hipLaunchKernelGGL((tsk::k_sym_split_mid<R>), dim3(tab->B, L, M / 256), dim3(256), 0, st, a);
  TSK_TRY(check_launch("k_sym_split_mid"));
  hipLaunchKernelGGL((tsk::k_sym_split_out<R>), dim3(tab->B, L), dim3(NT), lds, st, a);
  return check_launch("k_sym_split_out");
}

// The FP32 read-off of T(I,u,u) for L vectors on every sketch (mode 1: also
// lam_per = u . Re v).
tsk_status sym_power(tsk_ctx_t ctx, tsk_sym_tables_t tab, const float* S32, const float* s32, int L,
                     const float* U, float* V, double* lam_per, int mode, hipStream_t st) {
  if (tab->logb == 15) return sym_power_split_t<2>(ctx, tab, S32, s32, L, U, V, lam_per, mode, st);
  if (tab->logb == 16) return sym_power_split_t<4>(ctx, tab, S32, s32, L, U, V, lam_per, mode, st);
  if (tsk::sym_power_lds(tab->logb, tab->n) > kMaxLds - 256)
    return tsk::fail(TSK_EUNSUPPORTED, "symmetric power step: n=%d too large for b=%d", tab->n, tab->b);
  const cx<float>* tw = nullptr;
  const cx<float>* tw2 = nullptr;
  TSK_TRY(get_tw<float>(ctx, tab->logb + 1, &tw, tsk::sym_threads(tab->logb)));
  TSK_TRY(get_tw<float>(ctx, tab->logb, &tw2, tsk::sym_threads(tab->logb)));
  tsk::SymPowerArgs a;
  const size_t cnt = (size_t)tab->B * tab->n;
  a.hq = tab->hq;
  a.srt1 = tab->srt;
  a.ord1 = tab->ord;
  a.srt2 = tab->srt + cnt;
  a.ord2 = tab->ord + cnt;
  a.n = tab->n;
  a.B = tab->B;
  a.S = reinterpret_cast<const cx<float>*>(S32);
  a.s = reinterpret_cast<const cx<float>*>(s32);
  a.tw = tw;
  a.tw2 = tw2;
  a.U = U;
  a.V = V;
  a.lam_per = lam_per;
  a.mode = mode;
  switch (tab->logb) {
    case 8: return launch_sym_power_t<8>(a, L, st);
    case 9: return launch_sym_power_t<9>(a, L, st);
    case 10: return launch_sym_power_t<10>(a, L, st);
    case 11: return launch_sym_power_t<11>(a, L, st);
    case 12: return launch_sym_power_t<12>(a, L, st);
    case 13: return launch_sym_power_t<13>(a, L, st);
    case 14: return launch_sym_power_t<14>(a, L, st);
    default: break;
  }
  return tsk::fail(TSK_EUNSUPPORTED, "symmetric power step: b=%d", tab->b);
}

}  // namespace

namespace {

// The fixed-point LDS build of the symmetric sketches into s64 (written, or
// added to with accumulate): the dense build's kernel over the entries
// i <= j <= k (the pairs i <= j as fibres, from k = j on) and 2b real bins
// per sketch.
template <typename TIn>
tsk_status sym_build_impl(tsk_ctx_t ctx, tsk_sym_tables_t tab, const TIn* T, double* s64, int accumulate,
                          hipStream_t st) {
  const int n = tab->n, b = tab->b, B = tab->B;
  const int b2 = 2 * b;
  const int nrange = b2 > 16384 ? b2 / 16384 : 1;
  const int br = b2 / nrange;
  int lbr = 0;
  while ((1 << lbr) < br) ++lbr;
  const int Bv = B * nrange;
  const size_t per_sketch = (size_t)br * 8;
  int G = nrange > 1 ? 1
                     : (int)std::min<size_t>({(size_t)B, (size_t)tsk::kBuildMaxG,
                                              (size_t)kBuildPoolLarge * 8 / per_sketch});
  const int ngroups = (Bv + G - 1) / G;
  G = (Bv + ngroups - 1) / ngroups;
  const bool small = (size_t)G * per_sketch <= (size_t)kBuildPoolSmall * 8;
  const long long npairs = (long long)n * (n + 1) / 2;
  int nslab = pick_nslab(npairs, ngroups, small);
  long long pps = (npairs + nslab - 1) / nslab;
  pps = (pps + 3) / 4 * 4;
  nslab = (int)((npairs + pps - 1) / pps);
  // codes of the pairs per sketch, made once per table set (see the dense build)
  const long long efs = (npairs + 4 + 3) / 4 * 4;
  if ((size_t)G * efs * 4 > (size_t)0x7fffffff)
    return tsk::fail(TSK_EUNSUPPORTED, "symmetric build: n=%d too large", n);
  if (!tab->ef) {
    void* d = nullptr;
    TSK_HIP(hipMalloc(&d, (size_t)B * efs * sizeof(uint32_t)));
    hipLaunchKernelGGL(tsk::k_pair_codes, dim3(grid_for((size_t)B * efs, 256)), dim3(256), 0, st, tab->hq, n, B,
                       efs, reinterpret_cast<uint32_t*>(d));
    if (check_launch("k_pair_codes") != TSK_OK || hipStreamSynchronize(st) != hipSuccess) {
      (void)hipFree(d);
      return tsk::fail(TSK_EHIP, "symmetric build: pair codes failed");
    }
    tab->ef = reinterpret_cast<uint32_t*>(d);
  }
  void* partial = nullptr;
  void* stime = nullptr;
  void* amax = nullptr;
  TSK_TRY(ws_get(ctx, WS_PARTIAL, (size_t)ngroups * nslab * G * br * sizeof(double), &partial));
  TSK_TRY(ws_get(ctx, WS_STIME, (size_t)B * b2 * sizeof(double), &stime));
  const size_t cnt = (size_t)n * n * n;
  const int nabs = absmax_blocks(cnt);
  TSK_TRY(ws_get(ctx, WS_AMAX, (size_t)nabs * sizeof(unsigned long long), &amax));
  hipLaunchKernelGGL(tsk::k_absmax<TIn>, dim3(nabs), dim3(256), 0, st, T, cnt,
                     reinterpret_cast<unsigned long long*>(amax));
  TSK_TRY(check_launch("k_absmax"));
  tsk::BuildArgs<TIn> a;
  a.T = T;
  a.n = n;
  a.b = b;
  a.B = B;
  a.G = G;
  a.nrange = nrange;
  a.lbr = lbr;
  a.t3 = tab->hq;
  a.t3s = n;
  a.ef = tab->ef;
  a.efs = efs;
  a.nfib = npairs;
  a.pairs_per_slab = pps;
  a.nslab = nslab;
  a.ngroups = ngroups;
  a.absmax = reinterpret_cast<const unsigned long long*>(amax);
  a.nabs = nabs;
  a.partial = reinterpret_cast<double*>(partial);
  const int nblk = 8 * ngroups * ((nslab + 7) / 8);
  TSK_TRY((launch_build<TIn, true>(small, nrange > 1, nblk, a, st)));
  hipLaunchKernelGGL(tsk::k_build_reduce, dim3(grid_for((size_t)B * b2, 256)), dim3(256), 0, st,
                     (const double*)partial, (double*)stime, b2, B, G, nslab, nrange, lbr);
  TSK_TRY(check_launch("k_build_reduce"));
  hipLaunchKernelGGL(tsk::k_add64, dim3(grid_for((size_t)B * b2, 256)), dim3(256), 0, st, s64,
                     (const double*)stime, (size_t)B * b2, accumulate ? 1 : 0);
  return check_launch("k_add64");
}

}  // namespace

extern "C" tsk_status tsk_sym_sketch_build_dense(tsk_ctx_t ctx, tsk_sym_tables_t tab, const void* T,
                                                 tsk_dtype dtype, double* s64, float* s32, double* S64,
                                                 float* S32, int accumulate, void* stream) {
  TSK_TRY(check_sym(tab, ctx, "tsk_sym_sketch_build_dense"));
  if (!T || !s64 || !S64) return tsk::fail(TSK_EINVAL, "tsk_sym_sketch_build_dense: null T, s64 or S64");
  if (dtype != TSK_F32 && dtype != TSK_F64) return tsk::fail(TSK_EINVAL, "tsk_sym_sketch_build_dense: dtype");
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  const int n = tab->n, b = tab->b, B = tab->B;
  const size_t cplx = (size_t)B * b;
  (void)n;
  if (dtype == TSK_F32) TSK_TRY(sym_build_impl<float>(ctx, tab, (const float*)T, s64, accumulate, st));
  else TSK_TRY(sym_build_impl<double>(ctx, tab, (const double*)T, s64, accumulate, st));
  if (s32) {
    hipLaunchKernelGGL(tsk::k_c64to32, dim3(grid_for(cplx, 256)), dim3(256), 0, st,
                       reinterpret_cast<const cx<double>*>(s64), reinterpret_cast<cx<float>*>(s32), cplx);
    TSK_TRY(check_launch("k_c64to32"));
  }
  return fft64_rows(ctx, tab->logb, reinterpret_cast<const cx<double>*>(s64), reinterpret_cast<cx<double>*>(S64),
                    reinterpret_cast<cx<float>*>(S32), B, false, st);
}

extern "C" tsk_status tsk_sym_contract_tiuu(tsk_ctx_t ctx, tsk_sym_tables_t tab, const float* S32,
                                            const float* s32, int L, const float* U, float* V, void* stream) {
  TSK_TRY(check_sym(tab, ctx, "tsk_sym_contract_tiuu"));
  if (!S32 || !s32 || !U || !V) return tsk::fail(TSK_EINVAL, "tsk_sym_contract_tiuu: null argument");
  if (L < 1 || L > 65535) return tsk::fail(TSK_EINVAL, "tsk_sym_contract_tiuu: L=%d", L);
  TSK_TRY(set_device(ctx));
  return sym_power(ctx, tab, S32, s32, L, U, V, nullptr, 0, S(stream));
}

extern "C" tsk_status tsk_sym_decompose(tsk_ctx_t ctx, tsk_sym_tables_t tab, double* s64, float* s32,
                                        double* S64, float* S32, int k, int L, int T, const double* u0,
                                        uint64_t seed, double* lam_out, double* U_out, int32_t* tau_out,
                                        int32_t* flags_out, void* stream) {
  TSK_TRY(check_sym(tab, ctx, "tsk_sym_decompose"));
  if (!s64 || !s32 || !S64 || !S32 || !lam_out || !U_out)
    return tsk::fail(TSK_EINVAL, "tsk_sym_decompose: null argument");
  if (k < 1 || k > tab->n) return tsk::fail(TSK_EINVAL, "tsk_sym_decompose: k=%d outside [1,n]", k);
  if (L < 1 || L > 65535 || T < 1) return tsk::fail(TSK_EINVAL, "tsk_sym_decompose: L=%d, T=%d", L, T);
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  const int n = tab->n, b = tab->b, B = tab->B;
  const size_t cplx = (size_t)B * b;
  // workspace: U0/U1 [L][n] f32, V [L][B][n] f32, lam_per [L][B], lam_med [L],
  // u_hat [n], lam64 [B], cs [B][3][b] c64 (count sketches, then spectra),
  // cube [B][b] c64, tmp [B][b] c64, u0 [k][L][n] f64, flags [k][L]
  auto r = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t szU = r((size_t)L * n * 4), szV = r((size_t)L * B * n * 4);
  const size_t szLP = r((size_t)L * B * 8), szLM = r((size_t)L * 8), szUH = r((size_t)n * 8), szL64 = r((size_t)B * 8);
  const size_t szCS = r(3 * cplx * 16), szC = r(cplx * 16), szU0 = u0 ? 0 : r((size_t)k * L * n * 8);
  const size_t szF = flags_out ? 0 : r((size_t)k * L * 4);
  const size_t total = 2 * szU + szV + szLP + szLM + szUH + szL64 + 2 * szCS + 2 * szC + szU0 + szF;
  void* base = nullptr;
  TSK_TRY(ws_get(ctx, WS_U, total, &base));
  char* p = (char*)base;
  char* const end = p + total;
  auto take = [&](size_t sz) { char* q = p; p += sz; return q; };
  float* Ub[2] = {(float*)take(szU), (float*)take(szU)};
  float* V = (float*)take(szV);
  double* lam_per = (double*)take(szLP);
  double* lam_med = (double*)take(szLM);
  double* u_hat = (double*)take(szUH);
  double* lam64 = (double*)take(szL64);
  cx<double>* cs = (cx<double>*)take(szCS);
  cx<double>* Uf = (cx<double>*)take(szCS);
  cx<double>* cube = (cx<double>*)take(szC);
  cx<double>* tmp = (cx<double>*)take(szC);
  double* u0w = u0 ? nullptr : (double*)take(szU0);
  int32_t* flags = flags_out ? flags_out : (int32_t*)take(szF);
  if (p > end) return tsk::fail(TSK_EHIP, "internal: symmetric decomposition workspace layout");
  const double* u0d = u0;
  if (!u0) {
    TSK_TRY(upload_start_vectors(seed, k, L, n, u0w, st));
    u0d = u0w;
  }
  hipLaunchKernelGGL(tsk::k_fill_u32, dim3(grid_for((size_t)k * L, 256)), dim3(256), 0, st,
                     reinterpret_cast<unsigned*>(flags), 0u, (size_t)k * L);
  TSK_TRY(check_launch("k_fill_u32"));
  const size_t LN = (size_t)L * n;
  for (int c = 0; c < k; ++c) {
    hipLaunchKernelGGL(tsk::k_cvt<float>, dim3(grid_for(LN, 256)), dim3(256), 0, st, u0d + (size_t)c * LN, Ub[0],
                       LN);
    TSK_TRY(check_launch("k_cvt"));
    int cu = 0;
    for (int t = 0; t < T; ++t) {
      TSK_TRY(sym_power(ctx, tab, S32, s32, L, Ub[cu], V, nullptr, 0, st));
      TSK_TRY(median_norm_launch<float>(V, Ub[cu], Ub[cu ^ 1], flags + (size_t)c * L, L, n, B, st));
      cu ^= 1;
    }
    TSK_TRY(sym_power(ctx, tab, S32, s32, L, Ub[cu], V, lam_per, 1, st));
    TSK_TRY(lam_median_launch(lam_per, lam_med, L, B, st));
    hipLaunchKernelGGL(tsk::k_select<float>, dim3(1), dim3(256), 0, st, (const double*)lam_med, L,
                       (const float*)Ub[cu], n, u_hat, U_out + (size_t)c * n, tau_out ? tau_out + c : nullptr);
    TSK_TRY(check_launch("k_select"));
    // lambda_hat = med_m Re <s, s_X(u_hat)> in FP64, then deflation by
    // lambda_hat (s_u * s_u * s_u) in both domains
    hipLaunchKernelGGL(tsk::k_fill_u32, dim3(grid_for(12 * cplx, 256)), dim3(256), 0, st,
                       reinterpret_cast<unsigned*>(cs), 0u, 12 * cplx);
    TSK_TRY(check_launch("k_fill_u32"));
    hipLaunchKernelGGL(tsk::k_sym_cs64, dim3(B, 3), dim3(256), 0, st, tab->srt, tab->ord, n, b, B,
                       (const double*)u_hat, cs);
    TSK_TRY(check_launch("k_sym_cs64"));
    TSK_TRY(fft64_rows(ctx, tab->logb, cs, Uf, nullptr, 3 * B, false, st));
    hipLaunchKernelGGL(tsk::k_sym_lam, dim3(B), dim3(1024), 0, st, (const cx<double>*)S64, (const cx<double>*)Uf,
                       b, lam64, cube);
    TSK_TRY(check_launch("k_sym_lam"));
    hipLaunchKernelGGL(tsk::k_median_scalar, dim3(1), dim3(64), 0, st, (const double*)lam64, B, lam_out + c);
    TSK_TRY(check_launch("k_median_scalar"));
    hipLaunchKernelGGL(tsk::k_sym_axpy, dim3(grid_for(cplx, 256)), dim3(256), 0, st,
                       reinterpret_cast<cx<double>*>(S64), reinterpret_cast<cx<float>*>(S32),
                       (const cx<double>*)cube, (const double*)(lam_out + c), 1.0, cplx);
    TSK_TRY(check_launch("k_sym_axpy"));
    TSK_TRY(fft64_rows(ctx, tab->logb, cube, tmp, nullptr, B, true, st));
    hipLaunchKernelGGL(tsk::k_sym_axpy, dim3(grid_for(cplx, 256)), dim3(256), 0, st,
                       reinterpret_cast<cx<double>*>(s64), reinterpret_cast<cx<float>*>(s32), (const cx<double>*)tmp,
                       (const double*)(lam_out + c), 1.0 / (double)b, cplx);
    TSK_TRY(check_launch("k_sym_axpy"));
  }
  return TSK_OK;
}

// =============================================================================
// Fast spectral LDA (Appendix D, Algorithm 3): whitening and recovery
// =============================================================================

namespace {

tsk_status jacobi_eig(const double* G, int k, double* E, double* d, hipStream_t st) {
  static std::atomic<uint64_t> configured{0};
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  const uint64_t bit = 1ull << (dev & 63);
  if (!(configured.load() & bit)) {
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_jacobi_eig),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 2 * 100 * 100 * 8));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL(tsk::k_jacobi_eig, dim3(1), dim3(256), (size_t)2 * k * k * 8, st, G, k, E, d);
  return check_launch("k_jacobi_eig");
}

}  // namespace

extern "C" tsk_status tsk_lda_whiten(tsk_ctx_t ctx, const int32_t* rowptr, const int32_t* col, const int32_t* cnt,
                                     int D, int V, int K, double alpha0, const double* Omega, int iters,
                                     double* W_out, double* sigma_out, void* stream) {
  if (!ctx || !rowptr || !Omega || !W_out || !sigma_out)
    return tsk::fail(TSK_EINVAL, "tsk_lda_whiten: null argument");
  if (K < 1 || K > 100 || V < K || D < 1 || iters < 0 || iters > 1000)
    return tsk::fail(TSK_EINVAL, "tsk_lda_whiten: K=%d (1..100, <= V=%d), D=%d, iters=%d", K, V, D, iters);
  if (!(alpha0 >= 0.0) || alpha0 > 1e300)
    return tsk::fail(TSK_EINVAL, "tsk_lda_whiten: alpha0=%g must be finite and >= 0", alpha0);
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  int32_t nnz = 0;
  TSK_HIP(hipMemcpyAsync(&nnz, rowptr + D, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TSK_HIP(hipStreamSynchronize(st));
  if (nnz < 0) return tsk::fail(TSK_EINVAL, "tsk_lda_whiten: rowptr[D]=%d < 0", nnz);
  if (nnz > 0 && (!col || !cnt)) return tsk::fail(TSK_EINVAL, "tsk_lda_whiten: null col or cnt");
  const int G = std::max(1, std::min(1024, (D + 255) / 256));
  const int per_q = (D + G - 1) / G;
  size_t sort_tmp = 0;
  TSK_HIP(word_sort_tmp(&sort_tmp, nnz, V, st));
  size_t off = 0;
  std::vector<size_t> offs;
  auto take = [&](size_t bytes) {
    offs.push_back(off);
    off += (bytes + 255) & ~(size_t)255;
  };
  const size_t VK = (size_t)V * K;
  take((size_t)D * K * 8);          // 0 P
  take((size_t)D * 8);              // 1 cd
  take((size_t)D * 8);              // 2 cpd
  take((size_t)D * 8);              // 3 invm
  take((size_t)G * (K + 1) * 8);    // 4 q partials
  take((size_t)K * 8);              // 5 q
  take(8);                          // 6 D_eff
  take((size_t)nnz * 8 + 8);        // 7 packed entries
  take((size_t)nnz * 8 + 8);        // 8 packed entries in word order
  take((size_t)nnz * 4 + 4);        // 9 sorted word ids
  take((size_t)nnz * 4 + 4);        // 10 documents in word order
  take(sort_tmp);                   // 11 sort scratch
  take((size_t)(V + 1) * 4);        // 12 colptr
  take(VK * 8);                     // 13 Y
  take(VK * 8);                     // 14 Q
  take((size_t)K * K * 8);          // 15 Gram
  take((size_t)K * K * 8);          // 16 eigenvectors
  take((size_t)K * 8);              // 17 eigenvalues
  take((size_t)nnz * 4 + 4);        // 18 counts in word order
  take((size_t)D * 16);             // 19 packed (cpd, invm) per document
  void* base = nullptr;
  TSK_TRY(ws_get(ctx, WS_LDA, off, &base));
  auto at = [&](int i) { return reinterpret_cast<char*>(base) + offs[i]; };
  double* P = (double*)at(0);
  double *cd = (double*)at(1), *cpd = (double*)at(2), *invm = (double*)at(3);
  double *qpart = (double*)at(4), *q = (double*)at(5), *deff = (double*)at(6);
  int32_t* colptr = (int32_t*)at(12);
  double *Y = (double*)at(13), *Q = (double*)at(14), *Gm = (double*)at(15), *E = (double*)at(16);
  double* dv = (double*)at(17);
  // documents and counts of the nonzeros in word order
  int32_t *sdoc = (int32_t*)at(10), *scnt = (int32_t*)at(18);
  TSK_TRY(word_order(rowptr, col, cnt, D, V, nnz, (unsigned long long*)at(7), (unsigned long long*)at(8),
                     (uint32_t*)at(9), at(11), sort_tmp, colptr, sdoc, scnt, st));
  // Yout = M2 X
  auto apply = [&](const double* X, double* Yout) -> tsk_status {
    hipLaunchKernelGGL(tsk::k_doc_project<double>, dim3(std::min((D + 15) / 16, 8192)), dim3(256), 0, st, rowptr,
                       col, cnt, D, K, X, P, cd, cpd, invm);
    TSK_TRY(check_launch("k_doc_project"));
    hipLaunchKernelGGL(tsk::k_doc_q_partial<double>, dim3(G), dim3(128), 0, st, (const double*)P,
                       (const double*)invm, D, K, per_q, qpart);
    hipLaunchKernelGGL(tsk::k_doc_q_final, dim3(K + 1), dim3(256), 0, st, (const double*)qpart, G, K, q, deff);
    TSK_TRY(check_launch("k_doc_q"));
    double2* wk = (double2*)at(19);
    hipLaunchKernelGGL(tsk::k_pack_doc_weights, dim3(grid_for((size_t)D, 256)), dim3(256), 0, st,
                       (const double*)cpd, (const double*)invm, D, wk);
    TSK_TRY(check_launch("k_pack_doc_weights"));
    hipLaunchKernelGGL(tsk::k_lda_m2_apply, dim3(std::min(V, 16384)), dim3(64), 0, st, (const int32_t*)sdoc,
                       (const int32_t*)scnt, (const int32_t*)colptr, (const double*)P, (const double2*)wk, X,
                       (const double*)q, (const double*)deff, alpha0, V, K, Yout);
    return check_launch("k_lda_m2_apply");
  };
  // Q = orth(Yin)
  auto orth = [&](const double* Yin, double* Qout) -> tsk_status {
    TSK_TRY(gram2(ctx, Yin, Yin, Gm, V, K, st));
    TSK_TRY(jacobi_eig(Gm, K, E, dv, st));
    hipLaunchKernelGGL(tsk::k_orth_apply, dim3(std::min(V, 8192)), dim3(128), 0, st, Yin, (const double*)E,
                       (const double*)dv, Qout, V, K);
    return check_launch("k_orth_apply");
  };
  TSK_TRY(apply(Omega, Y));
  for (int it = 0; it < iters; ++it) {
    TSK_TRY(orth(Y, Q));
    TSK_TRY(apply(Q, Y));
  }
  TSK_TRY(orth(Y, Q));
  TSK_TRY(apply(Q, Y));
  TSK_TRY(gram2(ctx, (const double*)Q, (const double*)Y, Gm, V, K, st));
  TSK_TRY(jacobi_eig(Gm, K, E, dv, st));
  hipLaunchKernelGGL(tsk::k_whiten_out, dim3(std::min(V, 8192)), dim3(128), 0, st, (const double*)Q,
                     (const double*)E, (const double*)dv, W_out, sigma_out, V, K);
  return check_launch("k_whiten_out");
}

extern "C" tsk_status tsk_lda_heldout(tsk_ctx_t ctx, const int32_t* rowptr, const int32_t* col,
                                      const int32_t* cnt, int D, int V, int K, const double* Phi,
                                      double* pi_out, double* ll_out, void* stream) {
  if (!ctx || !rowptr || !Phi || !pi_out || !ll_out)
    return tsk::fail(TSK_EINVAL, "tsk_lda_heldout: null argument");
  if (D < 1 || V < 1 || K < 1 || K > 128 || K > V)
    return tsk::fail(TSK_EINVAL, "tsk_lda_heldout: D=%d, V=%d, K=%d (1 <= K <= min(V, 128))", D, V, K);
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  int32_t nnz = 0;
  TSK_HIP(hipMemcpyAsync(&nnz, rowptr + D, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  TSK_HIP(hipStreamSynchronize(st));
  if (nnz < 0) return tsk::fail(TSK_EINVAL, "tsk_lda_heldout: rowptr[D]=%d < 0", nnz);
  if (nnz > 0 && (!col || !cnt)) return tsk::fail(TSK_EINVAL, "tsk_lda_heldout: null col or cnt");
  const size_t gb = ((size_t)K * K * 8 + 255) & ~(size_t)255;
  const size_t pb = ((size_t)D * K * 8 + 255) & ~(size_t)255;
  const size_t db = ((size_t)D * 8 + 255) & ~(size_t)255;
  void* base = nullptr;
  TSK_TRY(ws_get(ctx, WS_HELD, gb + pb + 3 * db, &base));
  double* Gm = (double*)base;
  double* P = (double*)((char*)base + gb);
  double* cd = (double*)((char*)base + gb + pb);
  double* cpd = (double*)((char*)base + gb + pb + db);
  double* invm = (double*)((char*)base + gb + pb + 2 * db);
  TSK_TRY(gram2(ctx, Phi, Phi, Gm, V, K, st));
  hipLaunchKernelGGL(tsk::k_doc_project<double>, dim3(std::min((D + 15) / 16, 8192)), dim3(256), 0, st, rowptr,
                     col, cnt, D, K, Phi, P, cd, cpd, invm);
  TSK_TRY(check_launch("k_doc_project"));
  const size_t lds = tsk::simplex_ls_lds_words(K) * sizeof(double);
  static std::atomic<uint64_t> configured{0};
  const uint64_t bit = 1ull << (ctx->device & 63);
  if (!(configured.load() & bit)) {
    // the kernel's static LDS (reduction scratch) stays below 1 KB
    TSK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&tsk::k_simplex_ls),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds - 1024));
    configured.fetch_or(bit);
  }
  hipLaunchKernelGGL(tsk::k_simplex_ls, dim3(std::min(D, 4096)), dim3(256), lds, st, (const double*)Gm,
                     (const double*)P, rowptr, col, cnt, Phi, D, K, 10 * K + 10, pi_out, ll_out);
  return check_launch("k_simplex_ls");
}

extern "C" tsk_status tsk_lda_recover(tsk_ctx_t ctx, int V, int K, int k, double alpha0, const double* W,
                                      const double* lam, const double* U, double* alpha_out, double* mu_out,
                                      void* stream) {
  if (!ctx || !W || !lam || !U || !alpha_out || !mu_out) return tsk::fail(TSK_EINVAL, "tsk_lda_recover: null argument");
  if (K < 1 || K > 100 || V < 1 || k < 1) return tsk::fail(TSK_EINVAL, "tsk_lda_recover: V=%d, K=%d, k=%d", V, K, k);
  TSK_TRY(set_device(ctx));
  hipStream_t st = S(stream);
  void* base = nullptr;
  const size_t kk = ((size_t)K * K * 8 + 255) & ~(size_t)255, kv = ((size_t)K * 8 + 255) & ~(size_t)255;
  const size_t tv = ((size_t)k * K * 8 + 255) & ~(size_t)255;
  TSK_TRY(ws_get(ctx, WS_LDAR, 2 * kk + kv + tv, &base));
  double* Gm = (double*)base;
  double* E = (double*)((char*)base + kk);
  double* dv = (double*)((char*)base + 2 * kk);
  double* t = (double*)((char*)base + 2 * kk + kv);
  TSK_TRY(gram2(ctx, W, W, Gm, V, K, st));
  TSK_TRY(jacobi_eig(Gm, K, E, dv, st));
  hipLaunchKernelGGL(tsk::k_lda_tvec, dim3(k), dim3(128), 0, st, (const double*)E, (const double*)dv, U, K, t);
  TSK_TRY(check_launch("k_lda_tvec"));
  hipLaunchKernelGGL(tsk::k_lda_mu, dim3((V + 255) / 256, k), dim3(256), 0, st, W, (const double*)t, lam, alpha0, V,
                     K, mu_out, alpha_out);
  return check_launch("k_lda_mu");
}
