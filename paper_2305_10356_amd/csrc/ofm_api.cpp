// C ABI of libofm: argument checking, handles, and the kernel sequence of
// every call.  See include/ofm.h for the contract of each entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "ofm_internal.hpp"

using namespace ofm;

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return ofm_from_hip(e_);     \
  } while (0)

#define OFMCHK(expr)                 \
  do {                               \
    ofm_status s_ = (expr);          \
    if (s_ != OFM_OK) return s_;     \
  } while (0)

static ofm_status ofm_from_hip(hipError_t e) {
  if (e == hipErrorOutOfMemory) return OFM_E_NOMEM;
  return OFM_E_HIP;
}

namespace {

template <typename T>
ofm_status dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? OFM_E_NOMEM : OFM_E_HIP;
  }
  return OFM_OK;
}

template <typename T>
void dev_free(T*& p) {
  if (p) (void)hipFree(reinterpret_cast<void*>(p));
  p = nullptr;
}

bool supported_k(int k, int precision) {
  if (precision == OFM_FP64) return k == 4 || k == 8 || k == 16 || k == 32;
  return k == 4 || k == 8 || k == 16 || k == 32 || k == 64;
}

int sc_total(int k) {
  switch (k) {
    case 4: return SC<4>::TOTAL;
    case 8: return SC<8>::TOTAL;
    case 16: return SC<16>::TOTAL;
    case 32: return SC<32>::TOTAL;
    case 64: return SC<64>::TOTAL;
  }
  return 0;
}

struct SCOff {
  int M, H, K, GG, GGP, BETA, ALPHA, COEF, NROOT, RELRES, FVAL;
};

template <int KP>
SCOff sc_off_t() {
  using S = SC<KP>;
  return SCOff{S::M, S::H, S::K, S::GG, S::GGP, S::BETA, S::ALPHA, S::COEF, S::NROOT, S::RELRES,
               S::FVAL};
}

SCOff sc_off(int k) {
  switch (k) {
    case 4: return sc_off_t<4>();
    case 8: return sc_off_t<8>();
    case 16: return sc_off_t<16>();
    case 32: return sc_off_t<32>();
    default: return sc_off_t<64>();
  }
}

}  // namespace

struct TileTable {
  int tr = 0;
  int32_t* dev = nullptr;
  int64_t ntiles = 0;
  bool xcd = false;   // grouped order: tiles [xt[x], xt[x+1]) belong to XCD slot x
  int32_t xt[9] = {};
};

struct ofm_laplacian_s {
  LaplacianDev g;
  TileTable tt[3];  // TR = 16, 32, 64
  TileTable ut[3];  // tiles of the upper-triangle copy (g.nu > 0)
  std::vector<double> host_deg;
};

struct ofm_workspace_s {
  ofm_laplacian lap = nullptr;
  int k = 0;
  ofm_opts opts{};
  int64_t n = 0;
  size_t esz = 0;
  void* V[2] = {nullptr, nullptr};
  void* G[2] = {nullptr, nullptr};
  void* AX = nullptr;
  void* AV = nullptr;   // A V^t kept for the recurrence of A X (opts.recur)
  bool ax_valid = false;  // AX holds A X^t of the current iterate (opts.recur)
  bool h_valid = false;   // sc.H holds X^T A X of the current iterate (f2 without recur)
  void* Xb = nullptr;   // BF16 copies gathered by the SpMMs (OFM_FP32_BF16X)
  void* Vb = nullptr;
  int prec = 0;         // arithmetic of the kernels: OFM_FP64 or OFM_FP32
  int cur = 0;
  double* sc = nullptr;
  double* partials = nullptr;
  size_t part_cap = 0;     // doubles of partials
  double* lvl2 = nullptr;
  int* status = nullptr;
  int* frozen = nullptr;   // set on the device when the residual met tol
  // captured solve chunks (opts.graph): one per buffer parity at chunk start
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t chunk[2] = {nullptr, nullptr};
  const void* chunk_x = nullptr;
  int64_t t = 0;
  int64_t last_check = -1;
  bool initialized = false;
  const TileTable* tiles = nullptr;
  const void* pk = nullptr;
  // tiles of the Laplacian's upper-triangle copy when the line search's
  // products with A V come from it (without the recurrence: diag(V^T A V) for
  // f1; V^T A V for f2 at k <= 32, with X^T A V = (AX)^T V in the V pass from
  // the A X the SpMM of X stores)
  const TileTable* utiles = nullptr;
  bool f2u = false;       // the f2 form above
  bool products = false;  // f2 at k >= 32 otherwise: A V stored, products in a pass
  bool hc = false;       // gathers with the hot/cold cache policy (opts.gather)
  // per-pass event timing
  unsigned timing = 0;   // bit i: record events around the kernels of pass i
  struct Pending {
    int kind;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double ms[OFM_NUM_PASSES] = {0};
  int64_t count[OFM_NUM_PASSES] = {0};
};

namespace {

hipEvent_t take_event(ofm_workspace ws) {
  if (!ws->pool.empty()) {
    hipEvent_t e = ws->pool.back();
    ws->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// run one launch, bracketed by events when timing is on
template <typename F>
hipError_t timed(ofm_workspace ws, int kind, hipStream_t s, F&& launch) {
  if (!((ws->timing >> kind) & 1u)) return launch();
  hipEvent_t a = take_event(ws), b = take_event(ws);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  ws->pending.push_back({kind, a, b});
  return hipSuccess;
}

int pass_kind(int mode) {
  switch (mode) {
    case kGF1:
    case kAXF2:
    case kGF2: return OFM_PASS_SPMM_X;
    case kGPassF2:
    case kGPassF1: return OFM_PASS_G;
    case kVPass:
    case kVPassE: return OFM_PASS_V;
    case kAVF1:
    case kAVF2:
    case kSF2: return OFM_PASS_SPMM_V;
    case kUpdate:
    case kUpdateR: return OFM_PASS_UPDATE;
    case kEF: return OFM_PASS_OTHER;
    default: return OFM_PASS_OTHER;
  }
}

}  // namespace

// device status word -> ofm_status, the most severe first
static int device_status(int st) {
  return (st & kStNonfinite) ? OFM_E_NONFINITE
         : (st & kStCholesky) ? OFM_E_NUMERIC
         : (st & kStNoRoot)   ? OFM_E_NO_ROOT
                              : OFM_OK;
}

static const char* kStatusNames[] = {"OFM_OK",          "OFM_E_INVALID_ARG", "OFM_E_SHAPE",
                                     "OFM_E_GRAPH",     "OFM_E_NONFINITE",   "OFM_E_NUMERIC",
                                     "OFM_E_HIP",       "OFM_E_NOMEM",       "OFM_E_UNSUPPORTED",
                                     "OFM_E_NO_ROOT"};

extern "C" const char* ofm_status_string(int status) {
  if (status > 0 || status < -9) return "OFM_E_UNKNOWN";
  return kStatusNames[-status];
}

extern "C" const char* ofm_version(void) { return "ofm-gfx950 0.1"; }

// ---------------------------------------------------------------------------
// Laplacian
// ---------------------------------------------------------------------------

static void free_lap(ofm_laplacian L) {
  if (!L) return;
  dev_free(L->g.deg);
  dev_free(L->g.dinv);
  dev_free(L->g.sched);
  dev_free(L->g.sptr);
  dev_free(L->g.pk32);
  dev_free(L->g.pk64);
  dev_free(L->g.usched);
  dev_free(L->g.usptr);
  dev_free(L->g.upk32);
  dev_free(L->g.upk64);
  for (auto& t : L->tt) dev_free(t.dev);
  for (auto& t : L->ut) dev_free(t.dev);
  delete L;
}

// Share of the rows, by entry count, whose gathers keep the default cache
// policy when a workspace gathers with the hot/cold policy: the rows of the
// other columns are loaded non-temporally so they do not evict the rows that
// are gathered often (on a power-law graph the top fifth of the rows receive
// over half of the gathers).
constexpr double kHotShare = 0.2;

static void build_tiles(const std::vector<int32_t>& sdeg, int tr, bool reorder, int64_t p0,
                        int64_t p1, std::vector<int32_t>& t) {
  // tiles of consecutive positions in [p0, p1): rows of degree >= kHeavyDeg
  // (first when rows are sorted by degree) form "heavy" tiles of at most tr
  // rows and kHeavyTileNnz entries, processed one row per wavefront; the rest
  // form tiles of tr rows.  The heavy flag is the sign bit.
  int64_t p = p0;
  if (reorder) {
    while (p < p1 && sdeg[p] >= kHeavyDeg) {
      const int64_t st = p;
      int64_t nz = 0;
      while (p < p1 && sdeg[p] >= kHeavyDeg && p - st < tr &&
             (p == st || nz + sdeg[p] <= kHeavyTileNnz)) {
        nz += sdeg[p];
        ++p;
      }
      t.push_back((int32_t)st | (int32_t)0x80000000);
    }
  }
  while (p < p1) {
    t.push_back((int32_t)p);
    p = std::min<int64_t>(p1, p + tr);
  }
}

// Row-processing order from a grouping of the nodes, laid out for the eight
// XCDs: groups, largest entry count first, each go to the slot with the least
// work so far (entries + rows); rows without a group follow, one at a time in
// descending entry count, to the least loaded slot.  A slot lists its rows of
// kHeavyDeg or more entries first, then its groups in the order they were
// assigned, then its rows without a group; each of these by entry count,
// descending (ties by row).  Two stable counting sorts: O(n + max count +
// number of groups).  slot_pos receives the first position of every slot.
static void grouped_order(const std::vector<int32_t>& hrp, const int32_t* grp, int64_t n,
                          std::vector<int32_t>& sched, int64_t slot_pos[9]) {
  auto cnt = [&](int64_t i) { return (int64_t)(hrp[i + 1] - hrp[i]); };
  int32_t mx = 0;
  int64_t ng = 0;
  for (int64_t i = 0; i < n; ++i) {
    mx = std::max(mx, (int32_t)cnt(i));
    ng = std::max<int64_t>(ng, (int64_t)grp[i] + 1);
  }
  // rows by entry count, descending, ties in row order
  std::vector<int32_t> bydeg(n);
  {
    std::vector<int64_t> slot((size_t)mx + 2, 0);
    for (int64_t i = 0; i < n; ++i) ++slot[(size_t)(mx - cnt(i)) + 1];
    for (int32_t c = 0; c <= mx; ++c) slot[(size_t)c + 1] += slot[c];
    for (int64_t i = 0; i < n; ++i) bydeg[(size_t)slot[(size_t)(mx - cnt(i))]++] = (int32_t)i;
  }
  std::vector<int64_t> gcost((size_t)ng, 0);
  for (int64_t i = 0; i < n; ++i)
    if (grp[i] >= 0) gcost[(size_t)grp[i]] += cnt(i) + 1;
  std::vector<int32_t> gorder((size_t)ng);
  std::iota(gorder.begin(), gorder.end(), 0);
  std::stable_sort(gorder.begin(), gorder.end(),
                   [&](int32_t a, int32_t b) { return gcost[(size_t)a] > gcost[(size_t)b]; });
  int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto least = [&] {
    int x = 0;
    for (int y = 1; y < 8; ++y)
      if (load[y] < load[x]) x = y;
    return x;
  };
  std::vector<int8_t> gslot((size_t)ng, -1);
  std::vector<int32_t> gseq;  // groups in assignment order
  gseq.reserve((size_t)ng);
  for (int32_t gi : gorder) {
    if (gcost[(size_t)gi] == 0) break;
    const int x = least();
    gslot[(size_t)gi] = (int8_t)x;
    load[x] += gcost[(size_t)gi];
    gseq.push_back(gi);
  }
  std::vector<int8_t> rslot((size_t)n);
  for (int64_t q = 0; q < n; ++q) {
    const int32_t i = bydeg[(size_t)q];
    if (grp[i] >= 0) {
      rslot[(size_t)i] = gslot[(size_t)grp[i]];
    } else {
      const int x = least();
      rslot[(size_t)i] = (int8_t)x;
      load[x] += cnt(i) + 1;
    }
  }
  // bucket of a row: within slot x, 0 = heavy, 1 + r = the r-th group of the
  // slot, last = no group
  std::vector<int64_t> gbucket((size_t)ng, 0);
  std::vector<int64_t> base(9, 0);
  {
    int64_t per[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int32_t gi : gseq) gbucket[(size_t)gi] = 1 + per[gslot[(size_t)gi]]++;
    for (int x = 0; x < 8; ++x) base[x + 1] = base[x] + per[x] + 2;
  }
  auto bucket = [&](int32_t i) -> int64_t {
    const int x = rslot[(size_t)i];
    if (cnt(i) >= kHeavyDeg) return base[x];
    if (grp[i] >= 0) return base[x] + gbucket[(size_t)grp[i]];
    return base[x + 1] - 1;
  };
  std::vector<int64_t> next((size_t)base[8] + 1, 0);
  for (int64_t i = 0; i < n; ++i) ++next[(size_t)bucket((int32_t)i) + 1];
  for (int64_t b = 0; b < base[8]; ++b) next[(size_t)b + 1] += next[(size_t)b];
  for (int x = 0; x <= 8; ++x) slot_pos[x] = next[(size_t)base[x]];
  for (int64_t q = 0; q < n; ++q) {
    const int32_t i = bydeg[(size_t)q];
    sched[(size_t)next[(size_t)bucket(i)]++] = i;
  }
}

static ofm_status build_laplacian(int64_t n, int64_t nnz, const int32_t* row_ptr,
                                  const int32_t* col_idx, const void* vals, int vals_dtype,
                                  unsigned flags, const int32_t* groups, hipStream_t stream,
                                  ofm_laplacian* out);

extern "C" ofm_status ofm_build_laplacian(int64_t n, int64_t nnz, const int32_t* row_ptr,
                                          const int32_t* col_idx, const void* vals,
                                          int vals_dtype, unsigned flags, hipStream_t stream,
                                          ofm_laplacian* out) {
  return build_laplacian(n, nnz, row_ptr, col_idx, vals, vals_dtype, flags, nullptr, stream, out);
}

extern "C" ofm_status ofm_grouped_order(int64_t n, const int32_t* host_row_ptr,
                                        const int32_t* host_groups, int32_t* host_order,
                                        int64_t* host_slot_start) {
  if (n <= 0 || n >= (int64_t(1) << 31) || !host_row_ptr || !host_groups || !host_order ||
      !host_slot_start)
    return OFM_E_INVALID_ARG;
  if (host_row_ptr[0] != 0) return OFM_E_GRAPH;
  for (int64_t i = 0; i < n; ++i) {
    if (host_row_ptr[i + 1] < host_row_ptr[i]) return OFM_E_GRAPH;
    if ((int64_t)host_groups[i] >= n) return OFM_E_INVALID_ARG;
  }
  std::vector<int32_t> hrp(host_row_ptr, host_row_ptr + n + 1);
  std::vector<int32_t> sched((size_t)n);
  grouped_order(hrp, host_groups, n, sched, host_slot_start);
  std::memcpy(host_order, sched.data(), (size_t)n * sizeof(int32_t));
  return OFM_OK;
}

extern "C" ofm_status ofm_build_laplacian_grouped(int64_t n, int64_t nnz, const int32_t* row_ptr,
                                                  const int32_t* col_idx, const void* vals,
                                                  int vals_dtype, unsigned flags,
                                                  const int32_t* host_groups,
                                                  hipStream_t stream, ofm_laplacian* out) {
  if (!out) return OFM_E_INVALID_ARG;
  *out = nullptr;
  if (!host_groups || (flags & OFM_LAP_NO_REORDER) || n <= 0) return OFM_E_INVALID_ARG;
  for (int64_t i = 0; i < n; ++i)
    if ((int64_t)host_groups[i] >= n) return OFM_E_INVALID_ARG;
  return build_laplacian(n, nnz, row_ptr, col_idx, vals, vals_dtype, flags, host_groups, stream,
                         out);
}

static ofm_status build_laplacian(int64_t n, int64_t nnz, const int32_t* row_ptr,
                                  const int32_t* col_idx, const void* vals_in, int vals_dtype,
                                  unsigned flags, const int32_t* groups, hipStream_t stream,
                                  ofm_laplacian* out) {
  if (!out) return OFM_E_INVALID_ARG;
  *out = nullptr;
  if (n <= 0 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx)) return OFM_E_INVALID_ARG;
  if (n >= (int64_t(1) << 31) || nnz >= (int64_t(1) << 31)) return OFM_E_SHAPE;
  if (flags & ~(OFM_LAP_VALIDATE | OFM_LAP_NO_REORDER | OFM_LAP_NO_UPPER))
    return OFM_E_INVALID_ARG;
  if (vals_in && vals_dtype != OFM_FP64 && vals_dtype != OFM_FP32) return OFM_E_INVALID_ARG;
  // FP32 weights are widened (exactly) to an FP64 copy that lives for the call
  double* vals64 = nullptr;
  if (vals_in && vals_dtype == OFM_FP32 && nnz > 0) {
    ofm_status ast = dev_alloc(&vals64, nnz);
    if (ast != OFM_OK) return ast;
    if (launch_convert(nnz, 1, vals_in, vals64, stream) != hipSuccess) {
      dev_free(vals64);
      return OFM_E_HIP;
    }
  }
  const double* vals = vals64 ? vals64 : static_cast<const double*>(vals_in);
  struct Drop {
    double*& p;
    ~Drop() { dev_free(p); }
  } drop_vals{vals64};
  auto* L = new ofm_laplacian_s();
  LaplacianDev& g = L->g;
  g.n = n;
  g.nnz = nnz;
  g.reorder = !(flags & OFM_LAP_NO_REORDER);
  (void)hipGetDevice(&g.device);
  int* dflags = nullptr;
  double* w64 = nullptr;
  double* parts = nullptr;
  const int64_t nb = (n + 255) / 256;
  ofm_status st = OFM_OK;
  auto fail = [&](ofm_status s) {
    dev_free(dflags);
    dev_free(w64);
    dev_free(parts);
    free_lap(L);
    return s;
  };
  if ((st = dev_alloc(&g.deg, n)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&g.dinv, n)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&dflags, 1)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&w64, nnz)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&parts, nb)) != OFM_OK) return fail(st);
  if (hipMemsetAsync(dflags, 0, sizeof(int), stream) != hipSuccess) return fail(OFM_E_HIP);
  if (launch_graph_check(n, nnz, row_ptr, col_idx, vals, g.deg, dflags, stream) != hipSuccess)
    return fail(OFM_E_HIP);
  int hflags = 0;
  if (hipMemcpyAsync(&hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(OFM_E_HIP);
  if (hflags & (1 | 2 | 4 | 32)) return fail(OFM_E_GRAPH);
  if (flags & OFM_LAP_VALIDATE) {
    if (launch_graph_symcheck(n, row_ptr, col_idx, vals, dflags, stream) != hipSuccess)
      return fail(OFM_E_HIP);
    if (hipMemcpyAsync(&hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, stream) !=
            hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail(OFM_E_HIP);
    if (hflags & 16) return fail(OFM_E_GRAPH);
  }
  if (launch_graph_weights(n, row_ptr, col_idx, vals, g.deg, g.dinv, w64, parts, stream) !=
      hipSuccess)
    return fail(OFM_E_HIP);
  std::vector<double> hparts(nb);
  std::vector<int32_t> hrp(n + 1);
  L->host_deg.resize(n);
  if (hipMemcpyAsync(hparts.data(), parts, nb * sizeof(double), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipMemcpyAsync(hrp.data(), row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost,
                     stream) != hipSuccess ||
      hipMemcpyAsync(L->host_deg.data(), g.deg, n * sizeof(double), hipMemcpyDeviceToHost,
                     stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return fail(OFM_E_HIP);
  double na = 0.0;
  for (double v : hparts) na += v;
  g.normA2 = na;
  // row-processing order: by number of entries, descending, ties in row order
  // (a counting sort over the entry counts: O(n + max count))
  std::vector<int32_t> sched(n);
  int64_t slot_pos[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (groups) {
    grouped_order(hrp, groups, n, sched, slot_pos);
  } else if (g.reorder) {
    int32_t mx = 0;
    for (int64_t i = 0; i < n; ++i) mx = std::max(mx, hrp[i + 1] - hrp[i]);
    std::vector<int64_t> slot((size_t)mx + 2, 0);  // slot[mx - count]: next position
    for (int64_t i = 0; i < n; ++i) ++slot[(size_t)(mx - (hrp[i + 1] - hrp[i])) + 1];
    for (int32_t c = 0; c <= mx; ++c) slot[(size_t)c + 1] += slot[c];
    for (int64_t i = 0; i < n; ++i)
      sched[(size_t)slot[(size_t)(mx - (hrp[i + 1] - hrp[i]))]++] = (int32_t)i;
  } else {
    std::iota(sched.begin(), sched.end(), 0);
  }
  std::vector<int32_t> sptr(n + 1), sdeg(n);
  sptr[0] = 0;
  for (int64_t p = 0; p < n; ++p) {
    sdeg[p] = hrp[sched[p] + 1] - hrp[sched[p]];
    sptr[p + 1] = sptr[p] + sdeg[p];
  }
  if ((st = dev_alloc(&g.sched, n)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&g.sptr, n + 1)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(reinterpret_cast<int64_t**>(&g.pk32), nnz)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(reinterpret_cast<double**>(&g.pk64), 2 * nnz)) != OFM_OK) return fail(st);
  if (hipMemcpyAsync(g.sched, sched.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipMemcpyAsync(g.sptr, sptr.data(), (n + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    return fail(OFM_E_HIP);
  // cold mark: rows with fewer entries than the top kHotShare of rows by
  // entry count (ties at the cut count as hot); none when every row ties
  {
    int32_t mx = 0;
    for (int64_t i = 0; i < n; ++i) mx = std::max(mx, hrp[i + 1] - hrp[i]);
    std::vector<int64_t> hist((size_t)mx + 1, 0);
    for (int64_t i = 0; i < n; ++i) ++hist[(size_t)(hrp[i + 1] - hrp[i])];
    const int64_t want = std::max<int64_t>(1, (int64_t)(kHotShare * (double)n));
    int64_t seen = 0;
    int32_t cut = mx;
    for (; cut > 0; --cut) {
      seen += hist[(size_t)cut];
      if (seen >= want) break;
    }
    g.cold_below = cut;
  }
  if (launch_graph_pack(n, g.sched, row_ptr, col_idx, w64, g.sptr, g.pk32, g.pk64, g.cold_below,
                        stream) != hipSuccess)
    return fail(OFM_E_HIP);
  const int trs[3] = {16, 32, 64};
  for (int i = 0; i < 3; ++i) {
    std::vector<int32_t> t;
    if (groups) {
      L->tt[i].xcd = true;
      for (int x = 0; x < 8; ++x) {
        L->tt[i].xt[x] = (int32_t)t.size();
        build_tiles(sdeg, trs[i], true, slot_pos[x], slot_pos[x + 1], t);
      }
      L->tt[i].xt[8] = (int32_t)t.size();
    } else {
      build_tiles(sdeg, trs[i], g.reorder, 0, n, t);
    }
    t.push_back((int32_t)n);
    L->tt[i].tr = trs[i];
    L->tt[i].ntiles = (int64_t)t.size() - 1;
    if ((st = dev_alloc(&L->tt[i].dev, t.size())) != OFM_OK) return fail(st);
    if (hipMemcpyAsync(L->tt[i].dev, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       stream) != hipSuccess)
      return fail(OFM_E_HIP);
  }
  // upper-triangle copy for the line searches (no self-loops): the rows with
  // entries in it, by that count (descending), or, on a grouped
  // Laplacian, in the grouped order with the same eight XCD slots
  if (g.reorder && !(flags & OFM_LAP_NO_UPPER) && nnz > 0) {
    int32_t* ucnt = nullptr;
    if ((st = dev_alloc(&ucnt, n)) != OFM_OK) return fail(st);
    std::vector<int32_t> hu(n);
    int loops = 0;
    const bool ok =
        hipMemsetAsync(dflags, 0, sizeof(int), stream) == hipSuccess &&
        launch_graph_upper_count(n, row_ptr, col_idx, ucnt, dflags, stream) == hipSuccess &&
        hipMemcpyAsync(hu.data(), ucnt, n * sizeof(int32_t), hipMemcpyDeviceToHost, stream) ==
            hipSuccess &&
        hipMemcpyAsync(&loops, dflags, sizeof(int), hipMemcpyDeviceToHost, stream) == hipSuccess &&
        hipStreamSynchronize(stream) == hipSuccess;
    dev_free(ucnt);
    if (!ok) return fail(OFM_E_HIP);
    if (!loops) {
      std::vector<int32_t> usched(n);
      int64_t nu = 0;
      int64_t upos[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      if (groups) {
        // the grouped order without the rows that have nothing above them
        for (int x = 0; x < 8; ++x) {
          upos[x] = nu;
          for (int64_t p = slot_pos[x]; p < slot_pos[x + 1]; ++p)
            if (hu[(size_t)sched[(size_t)p]] > 0) usched[(size_t)nu++] = sched[(size_t)p];
        }
        upos[8] = nu;
      } else {
        int32_t mx = 0;
        for (int64_t i = 0; i < n; ++i) mx = std::max(mx, hu[(size_t)i]);
        std::vector<int64_t> slot((size_t)mx + 2, 0);  // slot[mx - count]: next position
        for (int64_t i = 0; i < n; ++i) ++slot[(size_t)(mx - hu[(size_t)i]) + 1];
        for (int32_t c = 0; c <= mx; ++c) slot[(size_t)c + 1] += slot[c];
        for (int64_t i = 0; i < n; ++i)
          usched[(size_t)slot[(size_t)(mx - hu[(size_t)i])]++] = (int32_t)i;
        while (nu < n && hu[(size_t)usched[(size_t)nu]] > 0) ++nu;
      }
      std::vector<int32_t> usptr(nu + 1), udeg(nu);
      usptr[0] = 0;
      for (int64_t p = 0; p < nu; ++p) {
        udeg[p] = hu[(size_t)usched[(size_t)p]];
        usptr[p + 1] = usptr[p] + udeg[p];
      }
      g.nu = nu;
      g.nnzu = nu > 0 ? usptr[nu] : 0;
      if (nu > 0) {
        if ((st = dev_alloc(&g.usched, nu)) != OFM_OK) return fail(st);
        if ((st = dev_alloc(&g.usptr, nu + 1)) != OFM_OK) return fail(st);
        if ((st = dev_alloc(reinterpret_cast<int64_t**>(&g.upk32), g.nnzu)) != OFM_OK)
          return fail(st);
        if ((st = dev_alloc(reinterpret_cast<double**>(&g.upk64), 2 * g.nnzu)) != OFM_OK)
          return fail(st);
        if (hipMemcpyAsync(g.usched, usched.data(), nu * sizeof(int32_t), hipMemcpyHostToDevice,
                           stream) != hipSuccess ||
            hipMemcpyAsync(g.usptr, usptr.data(), (nu + 1) * sizeof(int32_t),
                           hipMemcpyHostToDevice, stream) != hipSuccess ||
            launch_graph_pack_upper(nu, g.usched, row_ptr, col_idx, w64, g.usptr, g.upk32,
                                    g.upk64, g.cold_below, stream) != hipSuccess)
          return fail(OFM_E_HIP);
        for (int i = 0; i < 3; ++i) {
          std::vector<int32_t> t;
          if (groups) {
            L->ut[i].xcd = true;
            for (int x = 0; x < 8; ++x) {
              L->ut[i].xt[x] = (int32_t)t.size();
              build_tiles(udeg, trs[i], true, upos[x], upos[x + 1], t);
            }
            L->ut[i].xt[8] = (int32_t)t.size();
          } else {
            build_tiles(udeg, trs[i], true, 0, nu, t);
          }
          t.push_back((int32_t)nu);
          L->ut[i].tr = trs[i];
          L->ut[i].ntiles = (int64_t)t.size() - 1;
          if ((st = dev_alloc(&L->ut[i].dev, t.size())) != OFM_OK) return fail(st);
          // the host arrays of this block end here: wait for their copies
          if (hipMemcpyAsync(L->ut[i].dev, t.data(), t.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, stream) != hipSuccess ||
              hipStreamSynchronize(stream) != hipSuccess)
            return fail(OFM_E_HIP);
        }
      }
    }
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return fail(OFM_E_HIP);
  dev_free(dflags);
  dev_free(w64);
  dev_free(parts);
  *out = L;
  return OFM_OK;
}

extern "C" ofm_status ofm_laplacian_destroy(ofm_laplacian lap) {
  if (!lap) return OFM_E_INVALID_ARG;
  free_lap(lap);
  return OFM_OK;
}

extern "C" ofm_status ofm_laplacian_upper(ofm_laplacian lap, int64_t* host_rows,
                                          int64_t* host_nnz) {
  if (!lap) return OFM_E_INVALID_ARG;
  if (host_rows) *host_rows = lap->g.nu;
  if (host_nnz) *host_nnz = lap->g.nnzu;
  return OFM_OK;
}

extern "C" ofm_status ofm_laplacian_info(ofm_laplacian lap, int64_t* host_n, int64_t* host_nnz,
                                         double* host_normA2, double* host_degrees) {
  if (!lap) return OFM_E_INVALID_ARG;
  if (host_n) *host_n = lap->g.n;
  if (host_nnz) *host_nnz = lap->g.nnz;
  if (host_normA2) *host_normA2 = lap->g.normA2;
  if (host_degrees)
    std::memcpy(host_degrees, lap->host_deg.data(), lap->g.n * sizeof(double));
  return OFM_OK;
}

static const TileTable* tiles_for(ofm_laplacian lap, int precision, int k) {
  const int tr = tile_rows(precision, k);
  for (auto& t : lap->tt)
    if (t.tr == tr) return &t;
  return nullptr;
}

static void fill_graph(PassArgs& a, ofm_laplacian lap, const TileTable* tt, int precision) {
  a.sched = lap->g.sched;
  a.sptr = lap->g.sptr;
  a.tiles = tt->dev;
  a.ntiles = tt->ntiles;
  a.pk = precision == OFM_FP64 ? lap->g.pk64 : lap->g.pk32;
  a.cold_below = lap->g.cold_below;
  a.xcd = tt->xcd ? 1 : 0;
  for (int x = 0; x < 9; ++x) a.xt[x] = tt->xt[x];
}

// Grid of an SpMM launch (a.nblocks, a.xr).  Grouped order: one workgroup per
// chunk of xcd_chunk(mode) tiles per wave of the largest slot, times 8 (the
// hardware dispatches workgroups in order and places workgroup b on XCD b % 8,
// so each XCD walks its slot front to back as workgroups retire), when the
// reduction scratch holds that many partial rows of nv (cap, in doubles); else
// kMaxBlocks workgroups striding over the slots a tile per wave at a time.
// Chunks: the passes that form the direction load the k x k coefficients into
// LDS in every workgroup and take 4 tiles per wave; the others 1 (measured on
// the 2M-node graph: 1 / 2 / 4 / 8 tiles gave 1000 / 930 / 910 / 943 us for
// the SpMM of X and 752 / 779 / 817 / 896 us for that of V).
static int xcd_chunk(int mode) {
  return (mode == kGF1 || mode == kGF2 || mode == kAXF2) ? 4 : 1;
}

static int64_t xcd_full_grid(const TileTable* tt, int precision, int k, int chunk) {
  if (!tt->xcd) return 0;
  const int64_t span = (int64_t)spmm_wpb(precision, k) * chunk;
  int64_t per = 1;
  for (int x = 0; x < 8; ++x)
    per = std::max<int64_t>(per, ((int64_t)tt->xt[x + 1] - tt->xt[x] + span - 1) / span);
  return 8 * per;
}

static void spmm_grid(PassArgs& a, const TileTable* tt, int precision, int k, int nv,
                      size_t cap) {
  a.xr = 1;
  if (!tt->xcd) {
    a.nblocks = pass_blocks(precision, k, tt->ntiles);
    return;
  }
  const int chunk = xcd_chunk(a.mode);
  const int64_t one = xcd_full_grid(tt, precision, k, chunk);
  if (nv == 0 || (size_t)one * (size_t)nv <= cap) {
    a.nblocks = (int)one;
    a.xr = chunk;
    return;
  }
  const int64_t w = spmm_wpb(precision, k);
  a.nblocks = (int)std::min<int64_t>(kMaxBlocks, 8 * ((tt->ntiles + 8 * w - 1) / (8 * w)));
}

extern "C" ofm_status ofm_apply_A(ofm_laplacian lap, int k, int precision, const void* Z, void* Y,
                                  hipStream_t stream) {
  if (!lap || !Z || !Y) return OFM_E_INVALID_ARG;
  if (precision != OFM_FP32 && precision != OFM_FP64) return OFM_E_INVALID_ARG;
  if (!supported_k(k, precision)) return OFM_E_SHAPE;
  if (Z == Y) return OFM_E_INVALID_ARG;
  const TileTable* tt = tiles_for(lap, precision, k);
  if (!tt) return OFM_E_UNSUPPORTED;
  PassArgs a;
  a.n = lap->g.n;
  a.k = k;
  a.mode = kApply;
  a.Z = Z;
  a.Y = Y;
  fill_graph(a, lap, tt, precision);
  spmm_grid(a, tt, precision, k, 0, 0);
  HIPCHK(launch_spmm(precision, k, a, stream));
  return OFM_OK;
}

// ---------------------------------------------------------------------------
// Workspace and the iteration
// ---------------------------------------------------------------------------

static void free_ws(ofm_workspace ws) {
  if (!ws) return;
  for (auto& p : ws->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ws->pool) (void)hipEventDestroy(e);
  for (int i = 0; i < 2; ++i) {
    if (ws->chunk[i]) (void)hipGraphExecDestroy(ws->chunk[i]);
  }
  if (ws->cap_stream) (void)hipStreamDestroy(ws->cap_stream);
  for (int i = 0; i < 2; ++i) {
    dev_free(ws->V[i]);
    dev_free(ws->G[i]);
  }
  dev_free(ws->AX);
  dev_free(ws->AV);
  dev_free(ws->Xb);
  dev_free(ws->Vb);
  dev_free(ws->sc);
  dev_free(ws->partials);
  dev_free(ws->lvl2);
  dev_free(ws->status);
  dev_free(ws->frozen);
  delete ws;
}

static bool is_f2(int v) { return v == OFM_F2 || v == OFM_TRI_F2; }

// f2 without the recurrence at k >= 32: the SpMM of V stores A V and a
// streaming pass forms X^T A V and V^T A V
static bool f2_products_pass(const ofm_opts& o, int k) {
  return (o.variant == OFM_F2 || o.variant == OFM_TRI_F2) && !o.recur && k >= 32;
}

// Blocks from which the gather policy is chosen by timing (smaller ones fit
// the caches and keep the default policy).
constexpr size_t kHcMinBytes = size_t(32) << 20;

// Times Y = A Z with the default and with the hot/cold gather policy on the
// workspace's own buffers (Z = V[0], zeroed; Y = AX), alternating the two,
// and reports whether hot/cold was faster by more than 3%.  Synchronizing.
static ofm_status choose_gather(ofm_workspace ws, bool* hc) {
  PassArgs a;
  a.n = ws->n;
  a.k = ws->k;
  a.mode = kApply;
  a.Z = ws->V[0];
  a.Y = ws->AX;
  fill_graph(a, ws->lap, ws->tiles, ws->prec);
  spmm_grid(a, ws->tiles, ws->prec, ws->k, 0, 0);
  if (hipMemset(ws->V[0], 0, (size_t)ws->n * ws->k * ws->esz) != hipSuccess)
    return OFM_E_HIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return OFM_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return OFM_E_HIP;
  }
  ofm_status st = OFM_OK;
  auto run = [&](bool with_hc, float* ms) {
    PassArgs b = a;
    b.flags = with_hc ? kFlagHC : 0;
    float t = 0.0f;
    if (hipEventRecord(e0, nullptr) != hipSuccess ||
        launch_spmm(ws->prec, ws->k, b, nullptr) != hipSuccess ||
        hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&t, e0, e1) != hipSuccess)
      st = OFM_E_HIP;
    if (ms) *ms += t;
  };
  float t_def = 0.0f, t_hc = 0.0f;
  run(false, nullptr);  // warm-up of both
  run(true, nullptr);
  for (int r = 0; r < 2 && st == OFM_OK; ++r) {
    run(false, &t_def);
    run(true, &t_hc);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != OFM_OK) return st;
  *hc = t_hc < 0.97f * t_def;
  return OFM_OK;
}

extern "C" ofm_status ofm_workspace_create(ofm_laplacian lap, int k, const ofm_opts* host_opts,
                                           ofm_workspace* out) {
  if (!out) return OFM_E_INVALID_ARG;
  *out = nullptr;
  if (!lap || !host_opts) return OFM_E_INVALID_ARG;
  const ofm_opts& o = *host_opts;
  if (o.variant < 0 || o.variant > 3) return OFM_E_INVALID_ARG;
  if (o.precision != OFM_FP32 && o.precision != OFM_FP64 && o.precision != OFM_FP32_BF16X)
    return OFM_E_INVALID_ARG;
  if (o.max_iter < 1 || o.check_every < 1) return OFM_E_INVALID_ARG;
  if (o.first_step != 0 && o.first_step != 1) return OFM_E_INVALID_ARG;
  if (o.restart != 0 && o.restart != 1) return OFM_E_INVALID_ARG;
  if (!std::isfinite(o.alpha0) || !(o.tol >= 0.0)) return OFM_E_INVALID_ARG;
  if (o.graph != 0 && o.graph != 1) return OFM_E_INVALID_ARG;
  if (o.recur != 0 && o.recur != 1) return OFM_E_INVALID_ARG;
  if (o.gather < 0 || o.gather > 2) return OFM_E_INVALID_ARG;
  if (!(o.freeze_eps >= 0.0) || !std::isfinite(o.freeze_eps)) return OFM_E_INVALID_ARG;
  const int prec = o.precision == OFM_FP64 ? OFM_FP64 : OFM_FP32;
  if (!supported_k(k, prec)) return prec == OFM_FP64 && k == 64 ? OFM_E_UNSUPPORTED : OFM_E_SHAPE;
  if (k > lap->g.n) return OFM_E_SHAPE;
  const TileTable* tt = tiles_for(lap, prec, k);
  if (!tt) return OFM_E_UNSUPPORTED;
  auto* ws = new ofm_workspace_s();
  ws->lap = lap;
  ws->k = k;
  ws->opts = o;
  ws->n = lap->g.n;
  ws->prec = prec;
  ws->esz = prec == OFM_FP64 ? 8 : 4;
  ws->tiles = tt;
  ws->pk = prec == OFM_FP64 ? lap->g.pk64 : lap->g.pk32;
  if (lap->g.nu > 0 && !o.recur && (!is_f2(o.variant) || k <= 32)) {
    for (auto& t : lap->ut)
      if (t.tr == tt->tr) ws->utiles = &t;
  }
  ws->f2u = ws->utiles != nullptr && is_f2(o.variant);
  ws->products = f2_products_pass(o, k) && !ws->f2u;
  const size_t blk = (size_t)ws->n * k * ws->esz;
  // widest partial row: the V pass with X^T A V, [P | C | diag V^T G | 0 | E]
  const int nvmax = 3 * k * k + 3 * k;
  const int ny = (kMaxBlocks + kFinChunk - 1) / kFinChunk;
  ofm_status st = OFM_OK;
  auto fail = [&](ofm_status s) {
    free_ws(ws);
    return s;
  };
  for (int i = 0; i < 2; ++i) {
    if ((st = dev_alloc(reinterpret_cast<char**>(&ws->V[i]), blk)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(reinterpret_cast<char**>(&ws->G[i]), blk)) != OFM_OK) return fail(st);
  }
  if ((st = dev_alloc(reinterpret_cast<char**>(&ws->AX), blk)) != OFM_OK) return fail(st);
  if ((o.recur || ws->products) &&
      (st = dev_alloc(reinterpret_cast<char**>(&ws->AV), blk)) != OFM_OK)
    return fail(st);
  if (o.precision == OFM_FP32_BF16X) {
    if ((st = dev_alloc(reinterpret_cast<char**>(&ws->Xb), blk / 2)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(reinterpret_cast<char**>(&ws->Vb), blk / 2)) != OFM_OK) return fail(st);
  }
  if ((st = dev_alloc(&ws->sc, sc_total(k))) != OFM_OK) return fail(st);
  // partial rows: kMaxBlocks of every layout, or, on a grouped Laplacian, the
  // full grid of the plain steps (3k per row) when that is more; lvl2 then
  // also holds the intermediate levels of the reduction
  ws->part_cap = (size_t)kMaxBlocks * nvmax;
  size_t lvl2_size = (size_t)ny * nvmax;
  if (const int64_t full = xcd_full_grid(tt, prec, k, 1)) {
    ws->part_cap = std::max(ws->part_cap, (size_t)full * 3 * k);
    lvl2_size = std::max(lvl2_size, ws->part_cap / kFinChunk + ws->part_cap / (kFinChunk * kFinChunk) +
                                         (size_t)(2 + kMaxBlocks / kFinChunk) * nvmax);
  }
  if ((st = dev_alloc(&ws->partials, ws->part_cap)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&ws->lvl2, lvl2_size)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&ws->status, 1)) != OFM_OK) return fail(st);
  if ((st = dev_alloc(&ws->frozen, 1)) != OFM_OK) return fail(st);
  // cleared on the null stream, which the library's non-blocking streams do
  // not wait for, and waited for alone: creating a workspace does not wait
  // for work in flight elsewhere on the device
  if (hipMemsetAsync(ws->sc, 0, sc_total(k) * sizeof(double), nullptr) != hipSuccess ||
      hipMemsetAsync(ws->status, 0, sizeof(int), nullptr) != hipSuccess ||
      hipMemsetAsync(ws->frozen, 0, sizeof(int), nullptr) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess)
    return fail(OFM_E_HIP);
  // gather policy: the hot/cold path addresses the block with 31-bit offsets
  const bool hc_ok = o.precision != OFM_FP32_BF16X && blk <= (size_t)0x7fffffff;
  if (o.gather == 2 && !hc_ok) return fail(OFM_E_UNSUPPORTED);
  ws->hc = o.gather == 2;
  if (o.gather == 0 && hc_ok && blk >= kHcMinBytes && lap->g.cold_below > 0) {
    bool hc = false;
    if ((st = choose_gather(ws, &hc)) != OFM_OK) return fail(st);
    ws->hc = hc;
  }
  *out = ws;
  return OFM_OK;
}

extern "C" ofm_status ofm_workspace_destroy(ofm_workspace ws) {
  if (!ws) return OFM_E_INVALID_ARG;
  free_ws(ws);
  return OFM_OK;
}

static PassArgs base_args(ofm_workspace ws, int mode, int flags) {
  PassArgs a;
  a.n = ws->n;
  a.k = ws->k;
  a.mode = mode;
  a.variant = ws->opts.variant;
  a.flags = flags;
  a.sc = ws->sc;
  a.partials = ws->partials;
  a.status = ws->status;
  a.nv = partial_nv(ws->k, mode, flags);
  return a;
}

static ofm_status finalize(ofm_workspace ws, const PassArgs& a, hipStream_t s) {
  if (a.nv == 0) return OFM_OK;
  // the update of the recurrence writes [M | H]: H goes to its own slot
  const bool split = a.mode == kUpdateR && (a.flags & kFlagH);
  const int kk = ws->k * ws->k;
  double* out2 = split ? ws->sc + sc_off(ws->k).H : nullptr;
  HIPCHK(timed(ws, OFM_PASS_REDUCE, s, [&] {
    return launch_finalize(ws->partials, a.nblocks, a.nv, ws->sc + partial_off(ws->k, a.mode),
                           ws->lvl2, s, split ? kk : a.nv, out2);
  }));
  return OFM_OK;
}

static ofm_status run_spmm(ofm_workspace ws, PassArgs& a, hipStream_t s) {
  fill_graph(a, ws->lap, ws->tiles, ws->prec);
  if (ws->hc) a.flags |= kFlagHC;
  spmm_grid(a, ws->tiles, ws->prec, ws->k, a.nv, ws->part_cap);
  HIPCHK(timed(ws, pass_kind(a.mode), s, [&] { return launch_spmm(ws->prec, ws->k, a, s); }));
  return finalize(ws, a, s);
}

// a kFlagUpper pass over the upper-triangle copy (same rows of Z, fewer
// entries, its own processing order)
static ofm_status run_spmm_upper(ofm_workspace ws, PassArgs& a, hipStream_t s) {
  const LaplacianDev& g = ws->lap->g;
  a.sched = g.usched;
  a.sptr = g.usptr;
  a.tiles = ws->utiles->dev;
  a.ntiles = ws->utiles->ntiles;
  a.pk = ws->prec == OFM_FP64 ? g.upk64 : g.upk32;
  a.cold_below = g.cold_below;
  a.xcd = ws->utiles->xcd ? 1 : 0;
  for (int x = 0; x < 9; ++x) a.xt[x] = ws->utiles->xt[x];
  if (ws->hc) a.flags |= kFlagHC;
  spmm_grid(a, ws->utiles, ws->prec, ws->k, a.nv, ws->part_cap);
  HIPCHK(timed(ws, pass_kind(a.mode), s, [&] { return launch_spmm(ws->prec, ws->k, a, s); }));
  return finalize(ws, a, s);
}

static ofm_status run_dense(ofm_workspace ws, PassArgs& a, hipStream_t s) {
  const int tr = tile_rows(ws->prec, ws->k);
  a.nblocks = pass_blocks(ws->prec, ws->k, (ws->n + tr - 1) / tr);
  HIPCHK(timed(ws, pass_kind(a.mode), s, [&] { return launch_dense(ws->prec, ws->k, a, s); }));
  return finalize(ws, a, s);
}

// may_freeze: a residual <= tol freezes X (inside the iteration only)
static hipError_t run_residual(ofm_workspace ws, hipStream_t s, bool may_freeze) {
  return timed(ws, OFM_PASS_RESIDUAL, s, [&] {
    return launch_residual(ws->k, ws->opts.variant, ws->lap->g.normA2, ws->sc, ws->status,
                           may_freeze ? ws->opts.tol : 0.0, may_freeze ? ws->frozen : nullptr, s);
  });
}

extern "C" ofm_status ofm_set_timing(ofm_workspace ws, unsigned pass_mask) {
  if (!ws) return OFM_E_INVALID_ARG;
  ws->timing = pass_mask & OFM_TIMING_ALL;
  return OFM_OK;
}

extern "C" ofm_status ofm_get_timing(ofm_workspace ws, double* host_ms, int64_t* host_count,
                                     int reset) {
  if (!ws) return OFM_E_INVALID_ARG;
  for (auto& p : ws->pending) {
    HIPCHK(hipEventSynchronize(p.b));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    ws->ms[p.kind] += ms;
    ws->count[p.kind] += 1;
    ws->pool.push_back(p.a);
    ws->pool.push_back(p.b);
  }
  ws->pending.clear();
  for (int i = 0; i < OFM_NUM_PASSES; ++i) {
    if (host_ms) host_ms[i] = ws->ms[i];
    if (host_count) host_count[i] = ws->count[i];
    if (reset) {
      ws->ms[i] = 0.0;
      ws->count[i] = 0;
    }
  }
  return OFM_OK;
}

// G = g(X) into G[cur] with the per-column sums; f2 variants go through AX.
static ofm_status direction(ofm_workspace ws, void* X, const void* Gp, const void* Vp, int check,
                            hipStream_t s) {
  const int restart = ws->opts.restart ? kFlagRestart : 0;
  if (ws->opts.recur) {
    // A X exactly when the recurrence has no valid A X or a residual is due,
    // then the direction from the stored A X
    if (check || !ws->ax_valid) {
      PassArgs a = base_args(ws, kAXF2, check ? kFlagCheck : 0);
      a.Z = X;
      a.Zg = ws->Xb;
      a.Y = ws->AX;
      OFMCHK(run_spmm(ws, a, s));
      if (check) HIPCHK(run_residual(ws, s, true));
      ws->ax_valid = true;
    }
    PassArgs b = base_args(ws, is_f2(ws->opts.variant) ? kGPassF2 : kGPassF1, restart);
    b.X = X;
    b.AX = ws->AX;
    b.G = ws->G[ws->cur];
    b.Gp = Gp;
    b.Vp = Vp;
    return run_dense(ws, b, s);
  }
  if (!is_f2(ws->opts.variant)) {
    PassArgs a = base_args(ws, kGF1, (check ? kFlagCheck : 0) | restart);
    a.Z = X;
    a.Zg = ws->Xb;
    a.G = ws->G[ws->cur];
    a.Gp = Gp;
    a.Vp = Vp;
    OFMCHK(run_spmm(ws, a, s));
    if (check) HIPCHK(run_residual(ws, s, true));
  } else if (ws->h_valid) {
    // H of this iterate is known (advanced by the line search of the last
    // step): the direction is formed in the epilogue of the SpMM; on residual
    // steps the same pass also forms H and K exactly, replacing the advanced H
    PassArgs a = base_args(ws, kGF2, (check ? kFlagCheck : 0) | restart);
    a.Z = X;
    a.Zg = ws->Xb;
    a.G = ws->G[ws->cur];
    a.Gp = Gp;
    a.Vp = Vp;
    a.Y = ws->f2u ? ws->AX : nullptr;  // X^T A V of the V pass reads it
    OFMCHK(run_spmm(ws, a, s));
    if (check) HIPCHK(run_residual(ws, s, true));
  } else {
    PassArgs a = base_args(ws, kAXF2, check ? kFlagCheck : 0);
    a.Z = X;
    a.Zg = ws->Xb;
    a.Y = ws->AX;
    OFMCHK(run_spmm(ws, a, s));
    if (check) HIPCHK(run_residual(ws, s, true));
    PassArgs b = base_args(ws, kGPassF2, restart);
    b.X = X;
    b.AX = ws->AX;
    b.G = ws->G[ws->cur];
    b.Gp = Gp;
    b.Vp = Vp;
    OFMCHK(run_dense(ws, b, s));
  }
  return OFM_OK;
}

// V pass, SpMM(V), line search and update for direction G[cur]
static ofm_status search_and_update(ofm_workspace ws, void* X, const void* Vp, bool first,
                                    hipStream_t s) {
  const int cur = ws->cur;
  PassArgs v = base_args(ws, ws->f2u ? kVPassE : kVPass,
                         (first ? kFlagFirst : 0) | (ws->opts.restart ? kFlagRestart : 0));
  v.G = ws->G[cur];
  v.Vp = Vp;
  v.V = ws->V[cur];
  v.Vb = ws->Vb;
  v.X = X;
  v.AX = ws->f2u ? ws->AX : nullptr;
  OFMCHK(run_dense(ws, v, s));
  if (ws->f2u) {
    // V^T A V from the upper-triangle copy (X^T A V came with the V pass)
    PassArgs w = base_args(ws, kSF2, 0);
    w.Z = ws->V[cur];
    w.Zg = ws->Vb;
    OFMCHK(run_spmm_upper(ws, w, s));
  } else if (ws->products) {
    // A V stored by the SpMM of the f1 form, then X^T A V and V^T A V in a
    // streaming pass (at k >= 32 the two FP64 products in the SpMM's epilogue
    // cost it more occupancy than the pass costs)
    PassArgs w = base_args(ws, kAVF1, 0);
    w.Z = ws->V[cur];
    w.Zg = ws->Vb;
    w.X = X;
    w.Y = ws->AV;
    OFMCHK(run_spmm(ws, w, s));
    PassArgs e = base_args(ws, kEF, 0);
    e.X = X;
    e.V = ws->V[cur];
    e.Z = ws->AV;
    OFMCHK(run_dense(ws, e, s));
  } else if (ws->utiles) {
    // diag(V^T A V) over the upper-triangle copy (half the gathers)
    PassArgs w = base_args(ws, kAVF1, kFlagUpper);
    w.Z = ws->V[cur];
    w.Zg = ws->Vb;
    OFMCHK(run_spmm_upper(ws, w, s));
  } else {
    PassArgs w = base_args(ws, is_f2(ws->opts.variant) ? kAVF2 : kAVF1, 0);
    w.Z = ws->V[cur];
    w.Zg = ws->Vb;
    w.X = X;
    w.Y = ws->opts.recur ? ws->AV : nullptr;
    OFMCHK(run_spmm(ws, w, s));
  }
  // f2 without the recurrence: the line search also advances H to the next
  // iterate, so the next direction needs no stored A X
  const bool adv_h = is_f2(ws->opts.variant) && !ws->opts.recur;
  HIPCHK(timed(ws, OFM_PASS_LINESEARCH, s, [&] {
    return launch_linesearch(ws->k, ws->opts.variant, first && ws->opts.first_step == 1,
                             ws->opts.alpha0, adv_h ? 1 : 0, ws->f2u ? 2 : ws->utiles ? 1 : 0, ws->sc,
                             ws->status, ws->frozen, ws->opts.freeze_eps, s);
  }));
  ws->h_valid = adv_h;
  if (ws->opts.recur) {
    // X += V diag(alpha), A X += A V diag(alpha); M (and H for f2) of the new X
    PassArgs u = base_args(ws, kUpdateR, is_f2(ws->opts.variant) ? kFlagH : 0);
    u.X = X;
    u.Xw = X;
    u.Xb = ws->Xb;
    u.V = ws->V[cur];
    u.Z = ws->AV;
    u.AX = ws->AX;
    u.Y = ws->AX;
    OFMCHK(run_dense(ws, u, s));
  } else {
    PassArgs u = base_args(ws, kUpdate, 0);
    u.X = X;
    u.Xw = X;
    u.Xb = ws->Xb;
    u.V = ws->V[cur];
    OFMCHK(run_dense(ws, u, s));
  }
  ws->cur ^= 1;
  ws->t += 1;
  return OFM_OK;
}

static ofm_status gram_m(ofm_workspace ws, const void* X, hipStream_t s) {
  PassArgs a = base_args(ws, kGramM, 0);
  a.X = X;
  a.Xb = ws->Xb;  // (re)creates the BF16 copy of X when the workspace keeps one
  return run_dense(ws, a, s);
}

extern "C" ofm_status ofm_init(ofm_workspace ws, void* X, hipStream_t stream) {
  if (!ws || !X) return OFM_E_INVALID_ARG;
  HIPCHK(hipMemsetAsync(ws->frozen, 0, sizeof(int), stream));
  ws->cur = 0;
  ws->t = 0;
  ws->last_check = -1;
  ws->ax_valid = false;
  ws->h_valid = false;
  OFMCHK(gram_m(ws, X, stream));
  OFMCHK(direction(ws, X, nullptr, nullptr, 0, stream));
  OFMCHK(search_and_update(ws, X, nullptr, true, stream));
  ws->initialized = true;
  return OFM_OK;
}

extern "C" ofm_status ofm_step(ofm_workspace ws, void* X, hipStream_t stream) {
  if (!ws || !X) return OFM_E_INVALID_ARG;
  if (!ws->initialized) return OFM_E_INVALID_ARG;
  const int prev = ws->cur ^ 1;
  const int check = (ws->t % ws->opts.check_every) == 0;
  OFMCHK(direction(ws, X, ws->G[prev], ws->V[prev], check, stream));
  if (check) ws->last_check = ws->t;
  OFMCHK(search_and_update(ws, X, ws->V[prev], false, stream));
  return OFM_OK;
}

static ofm_status read_stats(ofm_workspace ws, hipStream_t stream, ofm_stats* o) {
  const SCOff so = sc_off(ws->k);
  double rv[2] = {0.0, 0.0};
  int st = 0;
  HIPCHK(hipMemcpyAsync(rv, ws->sc + so.RELRES, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(&st, ws->status, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  o->iters = ws->t;
  o->relres = ws->last_check >= 0 ? rv[0] : -1.0;
  o->objective = rv[1];
  o->relres_iter = ws->last_check;
  o->status = device_status(st);
  o->converged = (ws->last_check >= 0 && ws->opts.tol > 0.0 && rv[0] <= ws->opts.tol) ? 1 : 0;
  o->gather = ws->hc ? 2 : 1;
  o->reserved = 0;
  return OFM_OK;
}

extern "C" ofm_status ofm_get_stats(ofm_workspace ws, hipStream_t stream, ofm_stats* host_out) {
  if (!ws || !host_out) return OFM_E_INVALID_ARG;
  OFMCHK(read_stats(ws, stream, host_out));
  return (ofm_status)host_out->status;
}

// The check_every updates that start at ws->t (a step index one past a
// multiple of check_every) captured into a HIP graph.  Host-side step state is
// rewound after the capture; the replay advances it.
static ofm_status capture_chunk(ofm_workspace ws, void* X, hipGraphExec_t* out) {
  const int ce = ws->opts.check_every;
  if (!ws->cap_stream)
    HIPCHK(hipStreamCreateWithFlags(&ws->cap_stream, hipStreamNonBlocking));
  const int64_t t0 = ws->t;
  const int cur0 = ws->cur;
  const int64_t lc0 = ws->last_check;
  const bool axv0 = ws->ax_valid;
  const bool hv0 = ws->h_valid;
  const unsigned timing = ws->timing;
  ws->timing = 0;
  hipGraph_t g = nullptr;
  ofm_status st = OFM_OK;
  if (hipStreamBeginCapture(ws->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = OFM_E_HIP;
  } else {
    for (int i = 0; i < ce && st == OFM_OK; ++i) st = ofm_step(ws, X, ws->cap_stream);
    if (hipStreamEndCapture(ws->cap_stream, &g) != hipSuccess && st == OFM_OK) st = OFM_E_HIP;
  }
  ws->t = t0;
  ws->cur = cur0;
  ws->last_check = lc0;
  ws->ax_valid = axv0;
  ws->h_valid = hv0;
  ws->timing = timing;
  if (st == OFM_OK && hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess)
    st = OFM_E_HIP;
  if (g) (void)hipGraphDestroy(g);
  return st;
}

static ofm_status run_chunk(ofm_workspace ws, void* X, hipStream_t stream) {
  const int ce = ws->opts.check_every;
  if (ws->chunk_x != X) {
    for (int i = 0; i < 2; ++i) {
      if (ws->chunk[i]) HIPCHK(hipGraphExecDestroy(ws->chunk[i]));
      ws->chunk[i] = nullptr;
    }
    ws->chunk_x = X;
  }
  hipGraphExec_t& e = ws->chunk[ws->cur];
  if (!e) OFMCHK(capture_chunk(ws, X, &e));
  HIPCHK(hipGraphLaunch(e, stream));
  // the chunk's one residual evaluation is at its step index divisible by ce
  ws->last_check = ((ws->t + ce - 1) / ce) * ce;
  ws->t += ce;
  ws->cur ^= (ce & 1);
  return OFM_OK;
}

// The solve loop; `stop` (nullable) ends it at a residual check once nonzero.
static ofm_status solve_loop(ofm_workspace ws, void* X, hipStream_t stream, ofm_stats* host_out,
                             const std::atomic<int>* stop) {
  OFMCHK(ofm_init(ws, X, stream));
  ofm_stats st{};
  const int ce = ws->opts.check_every;
  while (ws->t < ws->opts.max_iter) {
    bool will_check;
    if (ws->opts.graph && ws->t % ce == 1 % ce && ws->t + ce <= ws->opts.max_iter) {
      OFMCHK(run_chunk(ws, X, stream));
      will_check = true;
    } else {
      will_check = (ws->t % ce) == 0;
      OFMCHK(ofm_step(ws, X, stream));
    }
    if (will_check) {
      OFMCHK(read_stats(ws, stream, &st));
      if (st.status != OFM_OK) break;
      if (st.converged) {
        // the step that found the residual below tol kept X (step size 0)
        ws->t = st.relres_iter;
        break;
      }
      if (stop && stop->load() != 0) break;
    }
  }
  OFMCHK(read_stats(ws, stream, &st));
  if (host_out) *host_out = st;
  return (ofm_status)st.status;
}

extern "C" ofm_status ofm_solve(ofm_workspace ws, void* X, hipStream_t stream,
                                ofm_stats* host_out) {
  if (!ws || !X) return OFM_E_INVALID_ARG;
  return solve_loop(ws, X, stream, host_out, nullptr);
}

extern "C" ofm_status ofm_residual(ofm_workspace ws, const void* X, hipStream_t stream,
                                   ofm_stats* host_out) {
  if (!ws || !X) return OFM_E_INVALID_ARG;
  OFMCHK(gram_m(ws, X, stream));
  PassArgs a = base_args(ws, kAXF2, kFlagCheck);
  a.Z = X;
  a.Y = ws->AX;
  OFMCHK(run_spmm(ws, a, stream));
  HIPCHK(run_residual(ws, stream, false));
  ws->last_check = ws->t;
  ws->ax_valid = false;
  ws->h_valid = false;  // the products above belong to the X passed in
  ofm_stats st{};
  OFMCHK(read_stats(ws, stream, &st));
  if (host_out) *host_out = st;
  return (ofm_status)st.status;
}

extern "C" ofm_status ofm_objective(ofm_workspace ws, const void* X, double* f_out, void* grad,
                                    hipStream_t stream) {
  if (!ws || !X || !f_out) return OFM_E_INVALID_ARG;
  if (ws->opts.variant == OFM_TRI_F1 || ws->opts.variant == OFM_TRI_F2) return OFM_E_UNSUPPORTED;
  ws->ax_valid = false;  // the products below overwrite A X
  ws->h_valid = false;   // and X^T A X
  // without a caller buffer the gradient goes to the current-direction slot,
  // which the next step overwrites anyway (the CG state is in the other slot)
  void* gout = grad ? grad : ws->G[ws->cur];
  OFMCHK(gram_m(ws, X, stream));
  if (ws->opts.variant == OFM_F1) {
    // the residual variant of the pass also forms X^T A X for the objective
    PassArgs a = base_args(ws, kGF1, kFlagCheck);
    a.Z = X;
    a.G = gout;
    OFMCHK(run_spmm(ws, a, stream));
  } else {
    PassArgs a = base_args(ws, kAXF2, 0);
    a.Z = X;
    a.Y = ws->AX;
    OFMCHK(run_spmm(ws, a, stream));
    PassArgs b = base_args(ws, kGPassF2, 0);
    b.X = X;
    b.AX = ws->AX;
    b.G = gout;
    OFMCHK(run_dense(ws, b, stream));
  }
  HIPCHK(timed(ws, OFM_PASS_OTHER, stream, [&] {
    return launch_objective(ws->k, ws->opts.variant, ws->lap->g.normA2, ws->sc, f_out, stream);
  }));
  return OFM_OK;
}

extern "C" ofm_status ofm_get_state(ofm_workspace ws, void* V_prev, void* G_prev,
                                    hipStream_t stream) {
  if (!ws || !V_prev || !G_prev) return OFM_E_INVALID_ARG;
  if (!ws->initialized) return OFM_E_INVALID_ARG;
  const int prev = ws->cur ^ 1;
  const size_t blk = (size_t)ws->n * ws->k * ws->esz;
  HIPCHK(hipMemcpyAsync(V_prev, ws->V[prev], blk, hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipMemcpyAsync(G_prev, ws->G[prev], blk, hipMemcpyDeviceToDevice, stream));
  return OFM_OK;
}

extern "C" ofm_status ofm_set_state(ofm_workspace ws, const void* X, const void* V_prev,
                                    const void* G_prev, int64_t t, hipStream_t stream) {
  if (!ws || !X || !V_prev || !G_prev || t < 1) return OFM_E_INVALID_ARG;
  ws->cur = 0;
  const int prev = 1;
  const size_t blk = (size_t)ws->n * ws->k * ws->esz;
  HIPCHK(hipMemcpyAsync(ws->V[prev], V_prev, blk, hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipMemcpyAsync(ws->G[prev], G_prev, blk, hipMemcpyDeviceToDevice, stream));
  OFMCHK(gram_m(ws, X, stream));
  PassArgs a = base_args(ws, kGGP, 0);
  a.Gp = ws->G[prev];
  OFMCHK(run_dense(ws, a, stream));
  HIPCHK(hipMemsetAsync(ws->frozen, 0, sizeof(int), stream));
  ws->t = t;
  ws->last_check = -1;
  ws->ax_valid = false;
  ws->h_valid = false;
  ws->initialized = true;
  return OFM_OK;
}

extern "C" ofm_status ofm_get_step_info(ofm_workspace ws, double* host_alpha, double* host_beta,
                                        double* host_coef, int32_t* host_nroots,
                                        hipStream_t stream) {
  if (!ws) return OFM_E_INVALID_ARG;
  const SCOff so = sc_off(ws->k);
  const int k = ws->k;
  std::vector<double> nr(k);
  if (host_alpha)
    HIPCHK(hipMemcpyAsync(host_alpha, ws->sc + so.ALPHA, k * sizeof(double), hipMemcpyDeviceToHost, stream));
  if (host_beta)
    HIPCHK(hipMemcpyAsync(host_beta, ws->sc + so.BETA, k * sizeof(double), hipMemcpyDeviceToHost, stream));
  if (host_coef)
    HIPCHK(hipMemcpyAsync(host_coef, ws->sc + so.COEF, 4 * k * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipMemcpyAsync(nr.data(), ws->sc + so.NROOT, k * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  if (host_nroots)
    for (int i = 0; i < k; ++i) host_nroots[i] = (int32_t)nr[i];
  return OFM_OK;
}

template <int KP>
static int product_off(int which) {
  using S = SC<KP>;
  const int offs[7] = {S::M, S::H, S::K, S::P, S::C, S::E, S::F};
  return offs[which];
}

extern "C" ofm_status ofm_get_products(ofm_workspace ws, int which, double* host_kxk,
                                       hipStream_t stream) {
  if (!ws || !host_kxk || which < 0 || which > 6) return OFM_E_INVALID_ARG;
  int off = 0;
  switch (ws->k) {
    case 4: off = product_off<4>(which); break;
    case 8: off = product_off<8>(which); break;
    case 16: off = product_off<16>(which); break;
    case 32: off = product_off<32>(which); break;
    default: off = product_off<64>(which); break;
  }
  HIPCHK(hipMemcpyAsync(host_kxk, ws->sc + off, (size_t)ws->k * ws->k * sizeof(double),
                        hipMemcpyDeviceToHost, stream));
  HIPCHK(hipStreamSynchronize(stream));
  return OFM_OK;
}

// ---------------------------------------------------------------------------
// Post-processing
// ---------------------------------------------------------------------------

extern "C" ofm_status ofm_row_normalize(int64_t n, int k, int precision, const void* X, void* Y,
                                        hipStream_t stream) {
  if (n < 0 || k < 1 || k > 64 || !X || !Y) return n < 0 || !X || !Y ? OFM_E_INVALID_ARG : OFM_E_SHAPE;
  if (precision != OFM_FP32 && precision != OFM_FP64) return OFM_E_INVALID_ARG;
  if (n == 0) return OFM_OK;
  HIPCHK(launch_row_normalize(n, k, precision, X, Y, stream));
  return OFM_OK;
}

extern "C" ofm_status ofm_scale(int64_t count, int precision, const double* scale,
                                const void* X, void* Y, hipStream_t stream) {
  if (count < 0 || !scale || !X || !Y) return OFM_E_INVALID_ARG;
  if (precision != OFM_FP32 && precision != OFM_FP64) return OFM_E_INVALID_ARG;
  if (count == 0) return OFM_OK;
  HIPCHK(launch_scale(count, precision, scale, X, Y, stream));
  return OFM_OK;
}

extern "C" ofm_status ofm_kmeans_assign(int64_t n, int dim, int n_clusters, const float* Y,
                                        const float* centroids, int32_t* labels, float* dist2,
                                        hipStream_t stream) {
  if (n < 0 || !Y || !centroids || !labels) return OFM_E_INVALID_ARG;
  if (dim < 1 || dim > 64 || n_clusters < 1 || n_clusters > 1024) return OFM_E_SHAPE;
  if (n == 0) return OFM_OK;
  HIPCHK(launch_kmeans_assign(n, dim, n_clusters, Y, centroids, labels, dist2, stream));
  return OFM_OK;
}

// Device buffers of one K-means run (all caller- or library-owned, none
// allocated here).
struct KmeansBufs {
  float* d2 = nullptr;       // [n] squared distance to the nearest chosen centre
  int32_t* pick = nullptr;   // [1] index of the next centre
  double* sums = nullptr;    // [nbs] chunk totals of the running sums
  int32_t* prev = nullptr;   // [n] labels of the previous Lloyd iteration
  double* part = nullptr;    // [nbk][n_clusters][dim + 1] block partials
  float* cnew = nullptr;     // [n_clusters][dim] next centroids
  int* changed = nullptr;    // [1] label change count
};

static ofm_status kmeans_check(int64_t n, int dim, int n_clusters, const float* Y,
                               const double* host_uniforms, int max_iter, const int32_t* labels,
                               const float* centroids) {
  if (n <= 0 || !Y || !host_uniforms || !labels || !centroids || max_iter < 1)
    return OFM_E_INVALID_ARG;
  if (dim < 1 || dim > 64 || n_clusters < 1 || n_clusters > 1024) return OFM_E_SHAPE;
  if (n_clusters > n) return OFM_E_SHAPE;
  for (int c = 0; c < n_clusters; ++c)
    if (!(host_uniforms[c] >= 0.0 && host_uniforms[c] < 1.0)) return OFM_E_INVALID_ARG;
  return OFM_OK;
}

// k-means++ seeding, then Lloyd iterations (Algorithm 1 step 5), on the given
// buffers.  Synchronizing.
static ofm_status kmeans_run(int64_t n, int dim, int n_clusters, const float* Y,
                             const double* host_uniforms, int max_iter, int32_t* labels,
                             float* centroids, int32_t* host_iters, hipStream_t stream,
                             const KmeansBufs& b) {
  const int nbk = kmeans_blocks(n, n_clusters * (dim + 1));
  // k-means++ seeding
  int32_t first = (int32_t)std::min<int64_t>((int64_t)(host_uniforms[0] * (double)n), n - 1);
  HIPCHK(hipMemcpyAsync(b.pick, &first, sizeof(int32_t), hipMemcpyHostToDevice, stream));
  HIPCHK(launch_kmeans_copy_centre(dim, Y, b.pick, centroids, 0, stream));
  HIPCHK(launch_kmeans_mindist(n, dim, Y, centroids, b.d2, 1, b.sums, stream));
  for (int c = 1; c < n_clusters; ++c) {
    HIPCHK(launch_kmeans_pick(n, b.d2, host_uniforms[c], b.sums, b.pick, stream));
    HIPCHK(launch_kmeans_copy_centre(dim, Y, b.pick, centroids, c, stream));
    HIPCHK(launch_kmeans_mindist(n, dim, Y, centroids + (size_t)c * dim, b.d2, 0, b.sums, stream));
  }
  // Lloyd iterations
  int it = 0;
  for (; it < max_iter; ++it) {
    HIPCHK(launch_kmeans_assign(n, dim, n_clusters, Y, centroids, labels, nullptr, stream));
    if (it > 0) {
      int h = 0;
      HIPCHK(hipMemsetAsync(b.changed, 0, sizeof(int), stream));
      HIPCHK(launch_count_changes(n, labels, b.prev, b.changed, stream));
      HIPCHK(hipMemcpyAsync(&h, b.changed, sizeof(int), hipMemcpyDeviceToHost, stream));
      HIPCHK(hipStreamSynchronize(stream));
      if (h == 0) break;
    }
    HIPCHK(launch_kmeans_centroid_sums(n, dim, n_clusters, Y, labels, b.part, nbk, stream));
    HIPCHK(launch_kmeans_centroid_final(dim, n_clusters, b.part, nbk, centroids, b.cnew, stream));
    HIPCHK(hipMemcpyAsync(centroids, b.cnew, (size_t)n_clusters * dim * sizeof(float),
                          hipMemcpyDeviceToDevice, stream));
    HIPCHK(hipMemcpyAsync(b.prev, labels, n * sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
  }
  HIPCHK(hipStreamSynchronize(stream));
  if (host_iters) *host_iters = it;
  return OFM_OK;
}

extern "C" ofm_status ofm_kmeans(int64_t n, int dim, int n_clusters, const float* Y,
                                 const double* host_uniforms, int max_iter, int32_t* labels,
                                 float* centroids, int32_t* host_iters, hipStream_t stream) {
  OFMCHK(kmeans_check(n, dim, n_clusters, Y, host_uniforms, max_iter, labels, centroids));
  const int nbk = kmeans_blocks(n, n_clusters * (dim + 1));
  const int nbs = kmeans_pick_chunks(n);
  KmeansBufs b;
  auto cleanup = [&]() {
    dev_free(b.d2);
    dev_free(b.pick);
    dev_free(b.sums);
    dev_free(b.prev);
    dev_free(b.part);
    dev_free(b.cnew);
    dev_free(b.changed);
  };
  ofm_status st = OFM_OK;
  if (st == OFM_OK) st = dev_alloc(&b.d2, n);
  if (st == OFM_OK) st = dev_alloc(&b.pick, 1);
  if (st == OFM_OK) st = dev_alloc(&b.sums, nbs);
  if (st == OFM_OK) st = dev_alloc(&b.prev, n);
  if (st == OFM_OK) st = dev_alloc(&b.part, (size_t)nbk * n_clusters * (dim + 1));
  if (st == OFM_OK) st = dev_alloc(&b.cnew, (size_t)n_clusters * dim);
  if (st == OFM_OK) st = dev_alloc(&b.changed, 1);
  if (st == OFM_OK)
    st = kmeans_run(n, dim, n_clusters, Y, host_uniforms, max_iter, labels, centroids, host_iters,
                    stream, b);
  if (st != OFM_OK) (void)hipStreamSynchronize(stream);  // nothing in flight uses b
  cleanup();
  return st;
}

// ---------------------------------------------------------------------------
// K-means without allocation: the buffers of a run live in one file-scope
// device array (each device holds its own copy for the life of the process);
// host code uses its address as hipGetSymbolAddress returns it per device.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[OFM_KMEANS_STATIC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// the array's device address on the current device, looked up once per device
ofm_status scratch_address(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return OFM_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return OFM_E_HIP;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return OFM_OK;
}
}  // namespace

extern "C" size_t ofm_kmeans_static_bytes(int64_t n, int dim, int n_clusters) {
  if (n <= 0 || dim < 1 || n_clusters < 1) return 0;
  const int nbk = kmeans_blocks(n, n_clusters * (dim + 1));
  const int nbs = kmeans_pick_chunks(n);
  return align256((size_t)nbk * n_clusters * (dim + 1) * sizeof(double)) +
         align256((size_t)nbs * sizeof(double)) + align256((size_t)n * sizeof(float)) +
         align256((size_t)n * sizeof(int32_t)) +
         align256((size_t)n_clusters * dim * sizeof(float)) + 2 * 256;
}

extern "C" ofm_status ofm_kmeans_noalloc(int64_t n, int dim, int n_clusters, const float* Y,
                                         const double* host_uniforms, int max_iter,
                                         int32_t* labels, float* centroids, int32_t* host_iters,
                                         hipStream_t stream) {
  OFMCHK(kmeans_check(n, dim, n_clusters, Y, host_uniforms, max_iter, labels, centroids));
  if (ofm_kmeans_static_bytes(n, dim, n_clusters) > (size_t)OFM_KMEANS_STATIC_BYTES)
    return OFM_E_SHAPE;
  void* base = nullptr;
  OFMCHK(scratch_address(&base));
  const int nbk = kmeans_blocks(n, n_clusters * (dim + 1));
  const int nbs = kmeans_pick_chunks(n);
  char* p = static_cast<char*>(base);
  KmeansBufs b;
  b.part = reinterpret_cast<double*>(p);
  p += align256((size_t)nbk * n_clusters * (dim + 1) * sizeof(double));
  b.sums = reinterpret_cast<double*>(p);
  p += align256((size_t)nbs * sizeof(double));
  b.d2 = reinterpret_cast<float*>(p);
  p += align256((size_t)n * sizeof(float));
  b.prev = reinterpret_cast<int32_t*>(p);
  p += align256((size_t)n * sizeof(int32_t));
  b.cnew = reinterpret_cast<float*>(p);
  p += align256((size_t)n_clusters * dim * sizeof(float));
  b.pick = reinterpret_cast<int32_t*>(p);
  p += 256;
  b.changed = reinterpret_cast<int*>(p);
  return kmeans_run(n, dim, n_clusters, Y, host_uniforms, max_iter, labels, centroids, host_iters,
                    stream, b);
}

extern "C" ofm_status ofm_gather_rows(int64_t nrows, int S, int row_floats, const int32_t* idx,
                                      const float* Z, int64_t zrows, float* Y,
                                      hipStream_t stream) {
  if (nrows < 0 || S < 1 || zrows < 1) return OFM_E_INVALID_ARG;
  if (row_floats != 16 && row_floats != 32 && row_floats != 64) return OFM_E_SHAPE;
  if (nrows == 0) return OFM_OK;
  if (!idx || !Z || !Y) return OFM_E_INVALID_ARG;
  (void)zrows;  // the caller guarantees 0 <= idx < zrows
  HIPCHK(launch_gather_rows(nrows, S, row_floats, idx, Z, Y, stream));
  return OFM_OK;
}

extern "C" ofm_status ofm_select_roots(int variant, int64_t count, const double* coef,
                                       double* alpha, int32_t* nroots, hipStream_t stream) {
  if (variant < 0 || variant > 3 || count < 0) return OFM_E_INVALID_ARG;
  if (count == 0) return OFM_OK;
  if (!coef || !alpha || !nroots) return OFM_E_INVALID_ARG;
  const int tri = (variant == OFM_TRI_F1 || variant == OFM_TRI_F2) ? 1 : 0;
  HIPCHK(launch_select_roots(tri, count, coef, alpha, nroots, stream));
  return OFM_OK;
}

// ---------------------------------------------------------------------------
// Batched solves
// ---------------------------------------------------------------------------

namespace {

// schedule candidates of a width group: c -> tiles per wavefront kBatchTpw[c % 4]
// (a graph's workers ~ its tiles / (waves per block x tpw)) with at most
// kBatchWorkers (c < 4) or half as many (c >= 4) workers per XCD
constexpr int kBatchCand = 8;
constexpr int kBatchWorkers = kBatchMaxWorkers;    // blocks per XCD
const int kBatchTpw[4] = {2, 4, 8, 16};
inline int cand_tpw(int c) { return kBatchTpw[c % 4]; }
inline int cand_workers(int c) { return c < 4 ? kBatchWorkers : kBatchWorkers / 2; }

struct BatchGroup {
  int k = 0;
  std::vector<int> idx;                 // members (batch indices)
  BatchGraph* dgraphs = nullptr;        // [n]
  int* dxlist = nullptr;                // members ordered by XCD
  int* dxoff = nullptr;                 // [9]
  std::vector<BatchGraph> hg;           // host copy of the descriptors
  int* active = nullptr;                // [n]
  int64_t* done = nullptr;              // [n]
  int* status = nullptr;                // [n]
  double* hist = nullptr;               // [n][kBatchHist]
  int* stalled = nullptr;               // [n]
  int64_t* tcount = nullptr;            // step counter of the group (device)
  double* sc = nullptr;                 // [n][SC total]
  double* partials = nullptr;
  double* lvl2 = nullptr;               // [n][workers / kFinChunk][nvmax]
  char* bufs = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;   // timing of the group's iterations (schedule)
  int chosen = 0;                         // schedule candidate in use
  double cand_ms[kBatchCand] = {};        // measured ms per iteration of every candidate
};

}  // namespace

constexpr int kFinishThreads = 4;  // concurrent FP64 finishing solves

struct ofm_batch_s {
  int count = 0;
  ofm_opts opts{};
  std::vector<ofm_laplacian> laps;
  std::vector<int> ks;
  std::vector<BatchGroup> groups;
  int fixed = -1;          // candidate set by ofm_batch_set_schedule (-1: timed)
  int wcap = 0;            // blocks per XCD below 64 set by ofm_batch_set_schedule (0: none)
  bool tuned = false;      // the groups' candidates were timed (kept for later solves)
  int escalated = 0;
  double loop_ms = 0.0;    // host time of the lockstep loop of the last solve
  double finish_ms = 0.0;  // host time of its FP64 finishing stage
  hipEvent_t start = nullptr;
  hipStream_t finish_streams[kFinishThreads] = {};
  // step state of the lockstep iteration (ofm_batch_init / ofm_batch_step)
  bool started = false;
  int cur = 0;             // ping-pong slot of the next direction
  int64_t t = 0;           // updates done
  int64_t last_check = -1;
  // check_every updates of every group captured as one HIP graph, per parity
  // of the ping-pong slot at the chunk's start, for the groups' schedule
  // candidates chunk_cand
  hipStream_t cap_stream = nullptr;
  hipEvent_t fork = nullptr;
  hipGraphExec_t chunk[2] = {nullptr, nullptr};
  std::vector<int> chunk_cand;
  int64_t replays = 0;     // chunks replayed by the last solve
  // persistent form of the lockstep loop (ofm_batch_set_persistent)
  bool persistent = false;
  unsigned* pbar = nullptr;  // [2] barrier words of the persistent launches
  int* perr = nullptr;       // set by a barrier wait that timed out
  int64_t plaunches = 0;     // persistent launches of the last solve
  int pworkers = 0;          // fewest workers per XCD a persistent launch used
  // copies of the starting blocks of the graphs that may be finished in FP64
  // (k <= 32, with a tolerance), taken when a solve starts: x0 + x0_off[i]
  float* x0 = nullptr;
  std::vector<int64_t> x0_off;  // -1: no copy
};

static void free_batch(ofm_batch b) {
  if (!b) return;
  dev_free(b->x0);
  dev_free(b->pbar);
  dev_free(b->perr);
  for (auto& e : b->chunk)
    if (e) (void)hipGraphExecDestroy(e);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto s : b->finish_streams)
    if (s) (void)hipStreamDestroy(s);
  for (auto& g : b->groups) {
    dev_free(g.dgraphs);
    dev_free(g.dxlist);
    dev_free(g.dxoff);
    dev_free(g.active);
    dev_free(g.done);
    dev_free(g.status);
    dev_free(g.hist);
    dev_free(g.stalled);
    dev_free(g.tcount);
    dev_free(g.sc);
    dev_free(g.partials);
    dev_free(g.lvl2);
    dev_free(g.bufs);
    if (g.stream) (void)hipStreamDestroy(g.stream);
    if (g.ev) (void)hipEventDestroy(g.ev);
    if (g.t0) (void)hipEventDestroy(g.t0);
    if (g.t1) (void)hipEventDestroy(g.t1);
  }
  if (b->start) (void)hipEventDestroy(b->start);
  delete b;
}

// graphs to XCDs, largest first onto the least loaded XCD (work ~ entries +
// rows); returns the graph order per XCD and the XCD offsets
static void batch_assign(const std::vector<double>& work, std::vector<int>& xlist,
                         std::vector<int>& xoff) {
  const int nx = 8;
  std::vector<int> order(work.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
  std::vector<std::vector<int>> per(nx);
  std::vector<double> load(nx, 0.0);
  for (int gi : order) {
    const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    per[x].push_back(gi);
    load[x] += work[gi];
  }
  xlist.clear();
  xoff.assign(nx + 1, 0);
  for (int x = 0; x < nx; ++x) {
    xoff[x] = (int)xlist.size();
    xlist.insert(xlist.end(), per[x].begin(), per[x].end());
  }
  xoff[nx] = (int)xlist.size();
}

extern "C" ofm_status ofm_batch_create(int count, const ofm_laplacian* host_laps,
                                       const int* host_ks, const ofm_opts* host_opts,
                                       ofm_batch* out) {
  if (!out) return OFM_E_INVALID_ARG;
  *out = nullptr;
  if (count < 1 || !host_laps || !host_ks || !host_opts) return OFM_E_INVALID_ARG;
  const ofm_opts& o = *host_opts;
  if (o.variant < 0 || o.variant > 3) return OFM_E_INVALID_ARG;
  if (o.precision != OFM_FP32 && o.precision != OFM_FP32_BF16X) return OFM_E_UNSUPPORTED;
  if (o.max_iter < 1 || o.check_every < 1 || !(o.tol >= 0.0)) return OFM_E_INVALID_ARG;
  if (o.first_step != 0 && o.first_step != 1) return OFM_E_INVALID_ARG;
  if ((o.restart | o.graph | o.recur) & ~1) return OFM_E_INVALID_ARG;
  static_assert(offsetof(ofm_opts, freeze_eps) == 56 && sizeof(ofm_opts) == 64,
                "ofm_opts layout is part of the ABI");
  if (o.gather < 0 || o.gather > 2) return OFM_E_INVALID_ARG;
  if (!(o.freeze_eps >= 0.0) || !std::isfinite(o.freeze_eps)) return OFM_E_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    if (!host_laps[i]) return OFM_E_INVALID_ARG;
    if (!supported_k(host_ks[i], OFM_FP32) || host_ks[i] > host_laps[i]->g.n) return OFM_E_SHAPE;
  }
  auto* B = new ofm_batch_s();
  B->count = count;
  B->opts = o;
  B->laps.assign(host_laps, host_laps + count);
  B->ks.assign(host_ks, host_ks + count);
  auto fail = [&](ofm_status s) {
    free_batch(B);
    return s;
  };
  if (hipEventCreate(&B->start) != hipSuccess) return fail(OFM_E_HIP);
  for (auto& fs : B->finish_streams)
    if (hipStreamCreateWithFlags(&fs, hipStreamNonBlocking) != hipSuccess) return fail(OFM_E_HIP);
  const int widths[5] = {4, 8, 16, 32, 64};
  const bool bf = o.precision == OFM_FP32_BF16X;
  for (int w : widths) {
    BatchGroup g;
    g.k = w;
    for (int i = 0; i < count; ++i)
      if (host_ks[i] == w) g.idx.push_back(i);
    if (g.idx.empty()) continue;
    B->groups.push_back(std::move(g));
  }
  for (auto& g : B->groups) {
    const int n = (int)g.idx.size();
    const int k = g.k;
    const int nvmax = 2 * k * k + 3 * k;
    const int sct = sc_total(k);
    ofm_status st;
    if (hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g.ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&g.t0) != hipSuccess || hipEventCreate(&g.t1) != hipSuccess)
      return fail(OFM_E_HIP);
    const int maxw = kBatchWorkers;
    size_t part_total = 0, buf_total = 0;
    std::vector<size_t> part_off(n), buf_off(n);
    std::vector<double> work(n);
    for (int m = 0; m < n; ++m) {
      ofm_laplacian L = host_laps[g.idx[m]];
      work[m] = (double)L->g.nnz * k + 8.0 * (double)L->g.n * k;
      part_off[m] = part_total;
      part_total += (size_t)maxw * nvmax;
      buf_off[m] = buf_total;
      const size_t blk = (size_t)L->g.n * k * 4;
      // V x2, G x2, AX (+ AV for the recurrence) (+ BF16 copies of X and V)
      buf_total += (o.recur ? 6 : 5) * blk + (bf ? blk : 0);
      buf_total = (buf_total + 255) & ~(size_t)255;
    }
    if ((st = dev_alloc(&g.active, n)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.done, n)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.status, n)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.hist, (size_t)n * kBatchHist)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.stalled, n)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.tcount, 1)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.sc, (size_t)n * sct)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.partials, part_total)) != OFM_OK) return fail(st);
    const size_t lvl2_per = (size_t)((kBatchWorkers + kFinChunk - 1) / kFinChunk) * nvmax;
    if ((st = dev_alloc(&g.lvl2, (size_t)n * lvl2_per)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.bufs, buf_total)) != OFM_OK) return fail(st);
    if (hipMemset(g.sc, 0, (size_t)n * sct * sizeof(double)) != hipSuccess) return fail(OFM_E_HIP);
    g.hg.resize(n);
    for (int m = 0; m < n; ++m) {
      ofm_laplacian L = host_laps[g.idx[m]];
      const TileTable* tt = tiles_for(L, OFM_FP32, k);
      BatchGraph& d = g.hg[m];
      d.n = L->g.n;
      d.sched = L->g.sched;
      d.sptr = L->g.sptr;
      d.tiles = tt->dev;
      d.ntiles = tt->ntiles;
      d.pk = L->g.pk32;
      if (L->g.nu > 0) {
        for (auto& ut : L->ut)
          if (ut.tr == tt->tr) {
            d.usched = L->g.usched;
            d.usptr = L->g.usptr;
            d.utiles = ut.dev;
            d.untiles = ut.ntiles;
            d.upk = L->g.upk32;
          }
      }
      const size_t blk = (size_t)L->g.n * k * 4;
      char* p = g.bufs + buf_off[m];
      d.V[0] = p;
      d.V[1] = p + blk;
      d.G[0] = p + 2 * blk;
      d.G[1] = p + 3 * blk;
      d.AX = p + 4 * blk;
      char* q = p + 5 * blk;
      d.AV = o.recur ? q : nullptr;
      if (o.recur) q += blk;
      d.Xb = bf ? q : nullptr;
      d.Vb = bf ? q + blk / 2 : nullptr;
      d.sc = g.sc + (size_t)m * sct;
      d.partials = g.partials + part_off[m];
      d.lvl2 = g.lvl2 + (size_t)m * lvl2_per;
      d.status = g.status + m;
      d.active = g.active + m;
      d.done_iter = g.done + m;
      d.hist = g.hist + (size_t)m * kBatchHist;
      d.stalled = g.stalled + m;
      d.normA2 = L->g.normA2;
    }
    std::vector<int> xlist, xoff;
    batch_assign(work, xlist, xoff);
    if ((st = dev_alloc(&g.dgraphs, n)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.dxlist, n)) != OFM_OK) return fail(st);
    if ((st = dev_alloc(&g.dxoff, 9)) != OFM_OK) return fail(st);
    if (hipMemcpy(g.dxlist, xlist.data(), n * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g.dxoff, xoff.data(), 9 * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
      return fail(OFM_E_HIP);
  }
  B->x0_off.assign(count, -1);
  if (o.tol > 0.0) {
    int64_t tot = 0;
    for (int i = 0; i < count; ++i)
      if (host_ks[i] <= 32) {
        B->x0_off[i] = tot;
        tot += ((host_laps[i]->g.n * host_ks[i] + 63) / 64) * 64;
      }
    if (tot > 0) {
      ofm_status st2 = dev_alloc(&B->x0, tot);
      if (st2 != OFM_OK) return fail(st2);
    }
  }
  *out = B;
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_destroy(ofm_batch b) {
  if (!b) return OFM_E_INVALID_ARG;
  free_batch(b);
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_schedule(ofm_batch b, int group, int* host_ngroups, int* host_k,
                                         int* host_tpw, int* host_workers, double* host_ms,
                                         int* host_escalated) {
  if (!b) return OFM_E_INVALID_ARG;
  if (host_ngroups) *host_ngroups = (int)b->groups.size();
  if (host_escalated) *host_escalated = b->escalated;
  if (group < 0 || group >= (int)b->groups.size()) return OFM_E_INVALID_ARG;
  const BatchGroup& g = b->groups[group];
  if (host_k) *host_k = g.k;
  if (host_tpw) *host_tpw = cand_tpw(g.chosen);
  if (host_workers)
    *host_workers = b->wcap > 0 ? std::min(b->wcap, cand_workers(g.chosen)) : cand_workers(g.chosen);
  if (host_ms)
    for (int c = 0; c < kBatchCand; ++c) host_ms[c] = g.cand_ms[c];
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_set_schedule(ofm_batch b, int tpw, int workers) {
  if (!b) return OFM_E_INVALID_ARG;
  if (tpw == 0) {
    b->fixed = -1;
    b->tuned = false;
    b->wcap = 0;
    return OFM_OK;
  }
  const int cap = (workers >= 8 && workers < 64) ? workers : 0;
  if (cap) workers = 64;
  for (int c = 0; c < kBatchCand; ++c)
    if (cand_tpw(c) == tpw && cand_workers(c) == workers) {
      b->wcap = cap;
      b->fixed = c;
      for (auto& g : b->groups) g.chosen = c;
      return OFM_OK;
    }
  return OFM_E_INVALID_ARG;
}

extern "C" ofm_status ofm_batch_phases(ofm_batch b, double* host_loop_ms, double* host_finish_ms,
                                       int64_t* host_replays) {
  if (!b) return OFM_E_INVALID_ARG;
  if (host_loop_ms) *host_loop_ms = b->loop_ms;
  if (host_finish_ms) *host_finish_ms = b->finish_ms;
  if (host_replays) *host_replays = b->replays;
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_set_persistent(ofm_batch b, int on) {
  if (!b || (on != 0 && on != 1)) return OFM_E_INVALID_ARG;
  if (on) {
    const ofm_opts& o = b->opts;
    if ((o.variant != OFM_F1 && o.variant != OFM_TRI_F1) || o.precision != OFM_FP32 || o.recur)
      return OFM_E_UNSUPPORTED;
    for (auto& g : b->groups)
      if (g.k > 32) return OFM_E_UNSUPPORTED;
    if (!b->pbar) OFMCHK(dev_alloc(&b->pbar, 2));
    if (!b->perr) OFMCHK(dev_alloc(&b->perr, 1));
  }
  b->persistent = on != 0;
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_persist_info(ofm_batch b, int64_t* host_launches,
                                             int* host_workers) {
  if (!b) return OFM_E_INVALID_ARG;
  if (host_launches) *host_launches = b->plaunches;
  if (host_workers) *host_workers = b->pworkers;
  return OFM_OK;
}

// FP64 solves of one graph that the FP32 loop did not finish, in three parts:
// the workspace and the FP64 block are made on the calling thread before the
// finishing threads start, so that the threads neither allocate, free nor
// synchronize the device; the solve runs on a thread's own stream; the result
// is written back to the graph's FP32 block on the calling thread after the
// threads have joined.
struct Finish {
  ofm_workspace ws = nullptr;
  double* X64 = nullptr;
};

static ofm_status finish_prepare(ofm_laplacian L, int k, const ofm_opts& o, int64_t used,
                                 Finish* f) {
  ofm_opts o64 = o;
  o64.precision = OFM_FP64;
  o64.max_iter = (int)(o.max_iter - used);
  o64.first_step = 0;
  o64.recur = 0;
  // eager steps: replayed as HIP graphs the finishing solves measured the same
  // (their time is the kernels of the slowest graph's iterations, not launches)
  o64.graph = 0;
  o64.gather = 1;  // no timing runs on the shared device
  OFMCHK(ofm_workspace_create(L, k, &o64, &f->ws));
  return dev_alloc(&f->X64, L->g.n * k);
}

// solve from the FP32 block src until converged, out of updates, or `claim`
// turns nonzero (the other solve of the same graph converged first); a
// converged solve claims the graph with `me` unless the other one has
static ofm_status finish_run(Finish& f, const void* src, hipStream_t s, ofm_stats* out,
                             std::atomic<int>* claim, int me) {
  if (claim->load() != 0) return OFM_OK;  // decided before this solve started
  const int64_t cnt = f.ws->n * f.ws->k;
  if (launch_convert(cnt, 1, src, f.X64, s) != hipSuccess) return OFM_E_HIP;
  const ofm_status es = solve_loop(f.ws, f.X64, s, out, claim);
  if (hipStreamSynchronize(s) != hipSuccess) return OFM_E_HIP;
  if (es == OFM_OK && out->converged) {
    int none = 0;
    claim->compare_exchange_strong(none, me);
  }
  return es;
}

static void finish_release(Finish& f) {
  dev_free(f.X64);
  if (f.ws) ofm_workspace_destroy(f.ws);
  f = Finish{};
}

// The FP64 finishing solves of a batched solve.  A graph that the FP32 loop
// leaves unconverged gets two solves that race: one continues from its FP32
// iterate (fast when the FP32 iteration stopped at its rounding floor), one
// restarts from its starting block (the FP32 rounding path can lead into a
// region where the iteration creeps, which an FP64 run from the start need not
// meet); the first to reach the tolerance wins and stops the other at its next
// residual check; with no winner the continued solve's result is kept.  The
// solves start once the FP32 loop has ended (run beside it, they slowed it by
// more than they gained).  kFinishThreads threads, each with a stream of its
// own, take the jobs in order.  Jobs live in a deque, whose elements keep
// their addresses as jobs are added.
struct FinishPool {
  enum : int { kContinue = 1, kRestart = 2 };
  struct Job {
    int graph = 0;
    int kind = kContinue;
    const void* src = nullptr;  // FP32 block the solve starts from
    ofm_stats st{};             // FP32 stats on entry
    ofm_stats s64{};            // the FP64 solve's
    ofm_status es = OFM_OK;
    Finish fin;
  };
  std::deque<Job> jobs;
  std::unique_ptr<std::atomic<int>[]> claim;  // per graph: 0, or the winning kind
  std::mutex mu;
  std::condition_variable cv;
  size_t next = 0;
  bool closed = false;
  std::vector<std::thread> threads;

  explicit FinishPool(int count) : claim(new std::atomic<int>[count]) {
    for (int i = 0; i < count; ++i) claim[i].store(0);
  }

  void start(int dev, const hipStream_t* streams) {
    for (int i = 0; i < kFinishThreads; ++i)
      threads.emplace_back([this, dev, s = streams[i]] {
        const bool on_device = hipSetDevice(dev) == hipSuccess;
        for (;;) {
          Job* jb = nullptr;
          {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [this] { return next < jobs.size() || closed; });
            if (next >= jobs.size()) return;
            jb = &jobs[next++];
          }
          jb->es = on_device ? finish_run(jb->fin, jb->src, s, &jb->s64, &claim[jb->graph], jb->kind)
                             : OFM_E_HIP;
        }
      });
  }
  // queue a prepared job (starts the threads on first use); false if the
  // threads cannot be started (the job is then released)
  bool push(Job&& j, int dev, const hipStream_t* streams) {
    try {
      if (threads.empty()) start(dev, streams);
      std::lock_guard<std::mutex> lk(mu);
      jobs.push_back(std::move(j));
    } catch (...) {
      finish_release(j.fin);
      return false;
    }
    cv.notify_one();
    return true;
  }
  void join() {
    {
      std::lock_guard<std::mutex> lk(mu);
      closed = true;
    }
    cv.notify_all();
    for (auto& t : threads) t.join();
    threads.clear();
  }
  ~FinishPool() {
    join();
    for (auto& j : jobs) finish_release(j.fin);
  }
};

// both finishing solves of graph i (FP32 stats st on entry, used updates done)
static ofm_status queue_finish(ofm_batch B, FinishPool& pool, int i, int k, const ofm_stats& st,
                               int dev, void* const* host_X) {
  for (int kind : {FinishPool::kContinue, FinishPool::kRestart}) {
    if (kind == FinishPool::kRestart && (!B->x0 || B->x0_off[i] < 0)) continue;
    FinishPool::Job jb;
    jb.graph = i;
    jb.kind = kind;
    jb.src = kind == FinishPool::kContinue ? host_X[i]
                                           : static_cast<const void*>(B->x0 + B->x0_off[i]);
    jb.st = st;
    const ofm_status ps = finish_prepare(B->laps[i], k, B->opts, st.iters, &jb.fin);
    if (ps != OFM_OK) {
      finish_release(jb.fin);
      return ps;
    }
    if (!pool.push(std::move(jb), dev, B->finish_streams)) return OFM_E_NOMEM;
  }
  return OFM_OK;
}

// the passes of one batched group: a dense or SpMM launch plus its per-graph
// reduction
static ofm_status bpass(BatchGroup& g, BatchArgs base, int mode, int flags, bool spmm) {
  BatchArgs a = base;
  a.mode = mode;
  a.flags = flags;
  a.nv = partial_nv(g.k, mode, flags);
  a.off = partial_off(g.k, mode);
  HIPCHK(spmm ? launch_batch_spmm(g.k, a, g.stream) : launch_batch_dense(g.k, a, g.stream));
  HIPCHK(launch_batch_finalize(a, g.stream));
  return OFM_OK;
}

static ofm_status batch_iteration(ofm_batch B, BatchGroup& g, int cur, int64_t t, bool first,
                                  bool check, int cand) {
  const ofm_opts& o = B->opts;
  BatchArgs base;
  base.k = g.k;
  base.variant = o.variant;
  base.cur = cur;
  base.bf16 = o.precision == OFM_FP32_BF16X;
  base.tol = o.tol;
  base.freeze_eps = o.freeze_eps;
  base.t = t;
  base.graphs = g.dgraphs;
  base.xlist = g.dxlist;
  base.xoff = g.dxoff;
  base.tcount = g.tcount;
  base.workers = B->wcap > 0 ? std::min(B->wcap, cand_workers(cand)) : cand_workers(cand);
  base.tpw = cand_tpw(cand);
  base.check_every = o.check_every;
  base.ngraphs = (int)g.idx.size();
  base.upper = (o.variant == OFM_F1 || o.variant == OFM_TRI_F1) && !o.recur;
  const int rs = o.restart ? kFlagRestart : 0;
  const int fs = first ? kFlagFirst : 0;
  if (first) OFMCHK(bpass(g, base, kGramM, 0, false));
  const bool f2 = o.variant == OFM_F2 || o.variant == OFM_TRI_F2;
  if (o.recur) {
    // A X exactly at the set-up step and when a residual is due, else by the
    // recurrence the previous update applied
    if (first || check) OFMCHK(bpass(g, base, kAXF2, check ? kFlagCheck : 0, true));
    if (check) HIPCHK(launch_batch_residual(g.k, base, g.stream));
    OFMCHK(bpass(g, base, f2 ? kGPassF2 : kGPassF1, rs | fs, false));
  } else {
    if (!f2) {
      OFMCHK(bpass(g, base, kGF1, (check ? kFlagCheck : 0) | rs | fs, true));
    } else {
      OFMCHK(bpass(g, base, kAXF2, check ? kFlagCheck : 0, true));
    }
    if (check) HIPCHK(launch_batch_residual(g.k, base, g.stream));
    if (f2) OFMCHK(bpass(g, base, kGPassF2, rs | fs, false));
  }
  OFMCHK(bpass(g, base, kVPass, rs | fs, false));
  OFMCHK(bpass(g, base, f2 ? kAVF2 : kAVF1, base.upper ? kFlagUpper : 0, true));
  HIPCHK(launch_batch_linesearch(g.k, base, o.alpha0, first && o.first_step == 1, g.stream));
  if (o.recur) {
    OFMCHK(bpass(g, base, kUpdateR, f2 ? kFlagH : 0, false));
  } else {
    OFMCHK(bpass(g, base, kUpdate, 0, false));
  }
  return OFM_OK;
}

// the group streams wait for the work enqueued so far on `stream`
static ofm_status batch_fork(ofm_batch B, hipStream_t stream) {
  HIPCHK(hipEventRecord(B->start, stream));
  for (auto& g : B->groups) HIPCHK(hipStreamWaitEvent(g.stream, B->start, 0));
  return OFM_OK;
}

// `stream` waits for the work enqueued so far on the group streams
static ofm_status batch_join(ofm_batch B, hipStream_t stream) {
  for (auto& g : B->groups) {
    HIPCHK(hipEventRecord(g.ev, g.stream));
    HIPCHK(hipStreamWaitEvent(stream, g.ev, 0));
  }
  return OFM_OK;
}

// Per-graph state reset and the set-up step of Algorithm 2 on every graph
// (on the group streams, after the work already on `stream`).
static ofm_status batch_start(ofm_batch B, void* const* host_X, hipStream_t stream) {
  for (int i = 0; i < B->count; ++i)
    if (!host_X[i]) return OFM_E_INVALID_ARG;
  OFMCHK(batch_fork(B, stream));
  for (auto& g : B->groups) {
    const int n = (int)g.idx.size();
    for (int m = 0; m < n; ++m) g.hg[m].X = host_X[g.idx[m]];
    std::vector<int> ones(n, 1);
    std::vector<int64_t> minus(n, -1);
    const int64_t zero = 0;
    HIPCHK(hipMemcpyAsync(g.dgraphs, g.hg.data(), n * sizeof(BatchGraph), hipMemcpyHostToDevice,
                          g.stream));
    HIPCHK(hipMemcpyAsync(g.active, ones.data(), n * sizeof(int), hipMemcpyHostToDevice, g.stream));
    HIPCHK(hipMemcpyAsync(g.done, minus.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, g.stream));
    HIPCHK(hipMemcpyAsync(g.tcount, &zero, sizeof(int64_t), hipMemcpyHostToDevice, g.stream));
    HIPCHK(hipMemsetAsync(g.status, 0, n * sizeof(int), g.stream));
    HIPCHK(hipMemsetAsync(g.stalled, 0, n * sizeof(int), g.stream));
    HIPCHK(hipMemsetAsync(g.hist, 0, (size_t)n * kBatchHist * sizeof(double), g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));  // the host vectors above go out of scope
  }
  B->cur = 0;
  B->t = 0;
  B->last_check = -1;
  for (auto& g : B->groups) OFMCHK(batch_iteration(B, g, B->cur, B->t, true, false, g.chosen));
  B->cur ^= 1;
  B->t = 1;
  B->started = true;
  return OFM_OK;
}

// one loop iteration of every group (eager, on the group streams) with
// schedule candidate cand, or each group's chosen one for cand < 0; timed:
// events around every group's launches
static ofm_status batch_step_groups(ofm_batch B, int cand, bool timed = false) {
  const bool check = (B->t % B->opts.check_every) == 0;
  for (auto& g : B->groups) {
    if (timed) HIPCHK(hipEventRecord(g.t0, g.stream));
    OFMCHK(batch_iteration(B, g, B->cur, B->t, false, check, cand < 0 ? g.chosen : cand));
    if (timed) HIPCHK(hipEventRecord(g.t1, g.stream));
  }
  if (check) B->last_check = B->t;
  B->cur ^= 1;
  B->t += 1;
  return OFM_OK;
}

// The check_every updates that start at B->t (one past a multiple of
// check_every; the last of them evaluates the residual) of every group,
// captured into one HIP graph: forked from a capture stream onto the group
// streams and joined back.  The host step state is rewound after the capture.
// Kernels read the step index from the groups' device counters, so one graph
// serves every chunk with the same parity of the ping-pong slot.
static ofm_status batch_capture(ofm_batch B, hipGraphExec_t* out) {
  if (!B->cap_stream)
    HIPCHK(hipStreamCreateWithFlags(&B->cap_stream, hipStreamNonBlocking));
  if (!B->fork) HIPCHK(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
  const int64_t t0 = B->t, lc0 = B->last_check;
  const int cur0 = B->cur;
  hipGraph_t graph = nullptr;
  ofm_status st = OFM_OK;
  if (hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return OFM_E_HIP;
  if (hipEventRecord(B->fork, B->cap_stream) != hipSuccess) st = OFM_E_HIP;
  for (auto& g : B->groups)
    if (st == OFM_OK && hipStreamWaitEvent(g.stream, B->fork, 0) != hipSuccess) st = OFM_E_HIP;
  for (int i = 0; i < B->opts.check_every && st == OFM_OK; ++i) st = batch_step_groups(B, -1);
  for (auto& g : B->groups) {
    if (st == OFM_OK && hipEventRecord(g.ev, g.stream) != hipSuccess) st = OFM_E_HIP;
    if (st == OFM_OK && hipStreamWaitEvent(B->cap_stream, g.ev, 0) != hipSuccess) st = OFM_E_HIP;
  }
  if (hipStreamEndCapture(B->cap_stream, &graph) != hipSuccess && st == OFM_OK) st = OFM_E_HIP;
  B->t = t0;
  B->cur = cur0;
  B->last_check = lc0;
  if (st == OFM_OK && hipGraphInstantiate(out, graph, nullptr, nullptr, 0) != hipSuccess)
    st = OFM_E_HIP;
  if (graph) (void)hipGraphDestroy(graph);
  return st;
}

// replay one chunk on `stream` (captured on first use), each group on its
// chosen schedule
static ofm_status batch_run_chunk(ofm_batch B, hipStream_t stream) {
  std::vector<int> key;
  for (auto& g : B->groups) key.push_back(g.chosen);
  if (B->chunk_cand != key) {
    for (auto& e : B->chunk) {
      if (e) HIPCHK(hipGraphExecDestroy(e));
      e = nullptr;
    }
    B->chunk_cand = key;
  }
  hipGraphExec_t& e = B->chunk[B->cur];
  if (!e) OFMCHK(batch_capture(B, &e));
  HIPCHK(hipGraphLaunch(e, stream));
  const int ce = B->opts.check_every;
  B->last_check = ((B->t + ce - 1) / ce) * ce;
  B->t += ce;
  B->cur ^= (ce & 1);
  ++B->replays;
  return OFM_OK;
}

// The check_every updates that start at B->t (as batch_run_chunk) as one
// persistent launch per width group, the groups one after another on
// `stream` (a cooperative launch needs its whole grid resident, so the groups
// do not share the chip).
static ofm_status batch_run_persistent(ofm_batch B, hipStream_t stream) {
  const ofm_opts& o = B->opts;
  const int rs = o.restart ? kFlagRestart : 0;
  for (auto& g : B->groups) {
    BatchArgs base;
    base.k = g.k;
    base.variant = o.variant;
    base.tol = o.tol;
    base.freeze_eps = o.freeze_eps;
    base.graphs = g.dgraphs;
    base.xlist = g.dxlist;
    base.xoff = g.dxoff;
    base.tcount = g.tcount;
    base.workers = B->wcap > 0 ? std::min(B->wcap, cand_workers(g.chosen)) : cand_workers(g.chosen);
    base.tpw = cand_tpw(g.chosen);
    base.check_every = o.check_every;
    base.ngraphs = (int)g.idx.size();
    base.upper = 1;
    BatchPersistArgs p;
    auto pass = [&](int which, int mode, int flags) {
      for (int c = 0; c < 2; ++c) {
        BatchArgs& a = p.pass[which][c];
        a = base;
        a.mode = mode;
        a.flags = flags;
        a.cur = c;
        a.nv = partial_nv(g.k, mode, flags);
        a.off = partial_off(g.k, mode);
      }
    };
    pass(kPGF1, kGF1, rs);
    pass(kPGF1C, kGF1, kFlagCheck | rs);
    pass(kPVPass, kVPass, rs);
    pass(kPAV, kAVF1, kFlagUpper);
    pass(kPUpdate, kUpdate, 0);
    p.t0 = B->t;
    p.cur0 = B->cur;
    p.steps = o.check_every;
    p.alpha0 = o.alpha0;
    p.bar = B->pbar;
    p.err = B->perr;
    HIPCHK(hipMemsetAsync(B->pbar, 0, 2 * sizeof(unsigned), stream));
    int used = 0;
    HIPCHK(launch_batch_persist(g.k, p, base.workers, &used, stream));
    B->pworkers = B->pworkers == 0 ? used : std::min(B->pworkers, used);
    ++B->plaunches;
  }
  const int ce = o.check_every;
  B->last_check = ((B->t + ce - 1) / ce) * ce;
  B->t += ce;
  B->cur ^= (ce & 1);
  return OFM_OK;
}

// 1 when any graph of the batch still iterates (synchronizing on `stream`,
// which must already be ordered after the work that set the flags)
static ofm_status batch_any_active(ofm_batch B, hipStream_t stream, int* any) {
  *any = 0;
  for (auto& g : B->groups) {
    std::vector<int> act(g.idx.size());
    HIPCHK(hipMemcpyAsync(act.data(), g.active, act.size() * sizeof(int), hipMemcpyDeviceToHost,
                          stream));
    HIPCHK(hipStreamSynchronize(stream));
    for (int a : act) *any |= a;
  }
  return OFM_OK;
}

static bool batch_locate(ofm_batch B, int i, BatchGroup** g, int* m) {
  for (auto& gr : B->groups)
    for (size_t j = 0; j < gr.idx.size(); ++j)
      if (gr.idx[j] == i) {
        *g = &gr;
        *m = (int)j;
        return true;
      }
  return false;
}

extern "C" ofm_status ofm_batch_init(ofm_batch B, void* const* host_X, hipStream_t stream) {
  if (!B || !host_X) return OFM_E_INVALID_ARG;
  OFMCHK(batch_start(B, host_X, stream));
  return batch_join(B, stream);
}

extern "C" ofm_status ofm_batch_step(ofm_batch B, hipStream_t stream) {
  if (!B) return OFM_E_INVALID_ARG;
  if (!B->started) return OFM_E_INVALID_ARG;
  OFMCHK(batch_fork(B, stream));
  OFMCHK(batch_step_groups(B, -1));
  return batch_join(B, stream);
}

extern "C" ofm_status ofm_batch_get_state(ofm_batch B, int i, void* V_prev, void* G_prev,
                                          hipStream_t stream) {
  if (!B || !V_prev || !G_prev || i < 0 || i >= B->count) return OFM_E_INVALID_ARG;
  if (!B->started) return OFM_E_INVALID_ARG;
  BatchGroup* g = nullptr;
  int m = 0;
  if (!batch_locate(B, i, &g, &m)) return OFM_E_INVALID_ARG;
  const int prev = B->cur ^ 1;
  const size_t blk = (size_t)g->hg[m].n * g->k * 4;
  HIPCHK(hipMemcpyAsync(V_prev, g->hg[m].V[prev], blk, hipMemcpyDeviceToDevice, stream));
  HIPCHK(hipMemcpyAsync(G_prev, g->hg[m].G[prev], blk, hipMemcpyDeviceToDevice, stream));
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_get_step_info(ofm_batch B, int i, double* host_alpha,
                                              double* host_beta, double* host_coef,
                                              int32_t* host_nroots, hipStream_t stream) {
  if (!B || i < 0 || i >= B->count) return OFM_E_INVALID_ARG;
  BatchGroup* g = nullptr;
  int m = 0;
  if (!batch_locate(B, i, &g, &m)) return OFM_E_INVALID_ARG;
  const int k = g->k;
  const SCOff so = sc_off(k);
  std::vector<double> sc(sc_total(k));
  HIPCHK(hipMemcpyAsync(sc.data(), g->hg[m].sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost,
                        stream));
  HIPCHK(hipStreamSynchronize(stream));
  for (int c = 0; c < k; ++c) {
    if (host_alpha) host_alpha[c] = sc[so.ALPHA + c];
    if (host_beta) host_beta[c] = sc[so.BETA + c];
    if (host_nroots) host_nroots[c] = (int32_t)sc[so.NROOT + c];
  }
  if (host_coef)
    for (int c = 0; c < 4 * k; ++c) host_coef[c] = sc[so.COEF + c];
  return OFM_OK;
}

extern "C" ofm_status ofm_batch_solve(ofm_batch B, void* const* host_X, hipStream_t stream,
                                      ofm_stats* host_stats) {
  if (!B || !host_X) return OFM_E_INVALID_ARG;
  for (int i = 0; i < B->count; ++i)
    if (!host_X[i]) return OFM_E_INVALID_ARG;
  const ofm_opts& o = B->opts;
  const int ce = o.check_every;
  const auto t_solve = std::chrono::steady_clock::now();
  // set-up step of Algorithm 2, then the loop.  Unless the schedule is fixed
  // or was timed by an earlier solve, the first iterations try the candidate
  // schedules (two iterations each, every group on the same candidate) and
  // keep the one whose iteration spans the least GPU time from the first
  // group's start to the last group's end (HIP events on the group streams,
  // the faster of the two iterations).  The groups share the chip, so a
  // group's own time under contention would favour schedules that only take
  // more of it from the others.
  B->replays = 0;
  B->plaunches = 0;
  B->pworkers = 0;
  if (B->persistent) HIPCHK(hipMemsetAsync(B->perr, 0, sizeof(int), stream));
  // the starting blocks of the graphs that may need a finishing solve
  if (B->x0)
    for (int i = 0; i < B->count; ++i)
      if (B->x0_off[i] >= 0)
        HIPCHK(hipMemcpyAsync(B->x0 + B->x0_off[i], host_X[i],
                              (size_t)B->laps[i]->g.n * B->ks[i] * sizeof(float),
                              hipMemcpyDeviceToDevice, stream));
  OFMCHK(batch_start(B, host_X, stream));
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  FinishPool pool(B->count);
  const bool tune = B->fixed < 0 && !B->tuned;
  const int64_t tune_end = tune ? 1 + 2 * kBatchCand : 0;
  bool on_stream = false;  // the loop runs as graph replays on `stream`
  while (B->t < o.max_iter) {
    const bool tuning = B->t < tune_end;
    const int cand = tuning ? (int)((B->t - 1) / 2) : -1;
    if (!tuning && (o.graph || B->persistent) && B->t % ce == 1 % ce &&
        B->t + ce <= o.max_iter) {
      if (!on_stream) {
        OFMCHK(batch_join(B, stream));
        on_stream = true;
      }
      if (B->persistent) OFMCHK(batch_run_persistent(B, stream));
      else OFMCHK(batch_run_chunk(B, stream));
      int any = 0;
      OFMCHK(batch_any_active(B, stream, &any));
      if (!any) break;
      continue;
    }
    if (on_stream) {
      OFMCHK(batch_fork(B, stream));
      on_stream = false;
    }
    const bool check = (B->t % ce) == 0;
    OFMCHK(batch_step_groups(B, cand, tuning));
    if (tuning) {
      const bool second = ((B->t - 2) % 2) == 1;  // B->t counts the step just enqueued
      double span = 0.0;
      for (auto& g : B->groups) {
        HIPCHK(hipEventSynchronize(g.t1));
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, B->groups[0].t0, g.t1));
        span = std::max(span, (double)ms);
      }
      for (auto& g : B->groups)
        g.cand_ms[cand] = second ? std::min(g.cand_ms[cand], span) : span;
      if (B->t == tune_end) {
        int best = 0;
        const double* ms = B->groups[0].cand_ms;
        for (int c = 1; c < kBatchCand; ++c)
          if (ms[c] < ms[best]) best = c;
        for (auto& g : B->groups) g.chosen = best;
        B->tuned = true;
      }
    }
    if (check) {
      OFMCHK(batch_join(B, stream));
      int any = 0;
      OFMCHK(batch_any_active(B, stream, &any));
      if (!any) break;
    }
  }
  if (on_stream) OFMCHK(batch_fork(B, stream));
  for (auto& g : B->groups) HIPCHK(hipStreamSynchronize(g.stream));
  if (B->persistent) {
    int err = 0;
    HIPCHK(hipMemcpy(&err, B->perr, sizeof(int), hipMemcpyDeviceToHost));
    if (err) return OFM_E_HIP;  // a grid barrier of a persistent launch timed out
  }
  const auto t_loop = std::chrono::steady_clock::now();
  B->loop_ms = std::chrono::duration<double, std::milli>(t_loop - t_solve).count();
  const int64_t t = B->t;
  const int64_t last_check = B->last_check;
  B->escalated = 0;
  // per-graph stats; a graph whose FP32 residual stopped decreasing before the
  // tolerance (or ran out of iterations) is finished in FP64
  std::vector<ofm_stats> all(B->count);
  for (auto& g : B->groups) {
    HIPCHK(hipStreamSynchronize(g.stream));
    const int n = (int)g.idx.size();
    const int sct = sc_total(g.k);
    const SCOff so = sc_off(g.k);
    std::vector<double> sc((size_t)n * sct);
    std::vector<int64_t> done(n);
    std::vector<int> stt(n), stl(n);
    HIPCHK(hipMemcpy(sc.data(), g.sc, sc.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(done.data(), g.done, n * sizeof(int64_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(stt.data(), g.status, n * sizeof(int), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(stl.data(), g.stalled, n * sizeof(int), hipMemcpyDeviceToHost));
    for (int m = 0; m < n; ++m) {
      ofm_stats st{};
      const double* s = sc.data() + (size_t)m * sct;
      st.iters = done[m] >= 0 ? done[m] : t;
      st.relres = last_check >= 0 ? s[so.RELRES] : -1.0;
      st.objective = s[so.FVAL];
      st.relres_iter = done[m] >= 0 ? done[m] : last_check;
      st.status = device_status(stt[m]);
      st.converged = (done[m] >= 0 && st.status == OFM_OK) ? 1 : 0;
      const bool escalate = !st.converged && st.status == OFM_OK && o.tol > 0.0 && g.k <= 32 &&
                            st.iters < o.max_iter;
      if (escalate) OFMCHK(queue_finish(B, pool, g.idx[m], g.k, st, dev, host_X));
      all[g.idx[m]] = st;  // replaced below for the finished graphs
    }
  }
  // the finishing solves (the batch's groups have completed: every group
  // stream was synchronized above)
  pool.join();
  for (auto& jb : pool.jobs)
    if (jb.es == OFM_E_HIP || jb.es == OFM_E_NOMEM || jb.es == OFM_E_INVALID_ARG ||
        jb.es == OFM_E_SHAPE || jb.es == OFM_E_UNSUPPORTED)
      return jb.es;
  // per finished graph: the winning solve, else the one continued from the
  // FP32 iterate; its FP64 block goes back to the graph's FP32 block
  for (auto& jb : pool.jobs) {
    const int won = pool.claim[jb.graph].load();
    if (won != 0 ? jb.kind != won : jb.kind != FinishPool::kContinue) continue;
    ofm_stats st = jb.st;
    if (jb.es == OFM_OK || jb.es == OFM_E_NONFINITE || jb.es == OFM_E_NUMERIC) {
      const ofm_stats& r = jb.s64;
      st.iters += r.iters;
      st.relres = r.relres;
      st.objective = r.objective;
      st.relres_iter = st.iters - r.iters + r.relres_iter;
      st.status = r.status;
      st.converged = r.converged;
      const int64_t cnt = jb.fin.ws->n * jb.fin.ws->k;
      HIPCHK(launch_convert(cnt, 0, jb.fin.X64, host_X[jb.graph], stream));
    }
    all[jb.graph] = st;
    ++B->escalated;
  }
  HIPCHK(hipStreamSynchronize(stream));
  B->finish_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_loop).count();
  if (host_stats)
    for (int i = 0; i < B->count; ++i) host_stats[i] = all[i];
  for (auto& g : B->groups) {
    HIPCHK(hipEventRecord(g.ev, g.stream));
    HIPCHK(hipStreamWaitEvent(stream, g.ev, 0));
  }
  return OFM_OK;
}
