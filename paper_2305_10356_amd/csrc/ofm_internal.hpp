// Internal declarations shared by the HIP translation units of libofm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ofm.h"

namespace ofm {

constexpr int kWave = 64;
constexpr int kHeavyDeg = 64;     // rows of at least this degree use a whole wave
constexpr int kHeavyTileNnz = 1024;
#ifndef OFM_MAX_BLOCKS
#define OFM_MAX_BLOCKS 1024
#endif
#ifndef OFM_GATHER_CH
#define OFM_GATHER_CH 8
#endif
constexpr int kMaxBlocks = OFM_MAX_BLOCKS;  // persistent grid cap for reduction kernels
constexpr int kGatherChunk = OFM_GATHER_CH; // entries in flight per lane group and pass
constexpr int kFinChunk = 32;     // partial rows summed per first-level finalize block

// Row-major N x KP tile geometry of a wave: each row is KP*sizeof(T) bytes,
// read as 16-byte vectors by LPR consecutive lanes; a wave handles RPW rows
// per pass and TR rows per tile (TR >= 16 for the 16-row MFMA sub-tiles).
template <typename T, int KP>
struct Geo {
  static constexpr int VECN = 16 / (int)sizeof(T);
  static constexpr int LPR = KP / VECN;
  static constexpr int RPW = kWave / LPR;
  static constexpr int TR = RPW > 16 ? RPW : 16;
  static constexpr int NPASS = TR / RPW;
  static constexpr int NSUB = TR / 16;
  static constexpr int LDST = KP + 1;           // LDS row stride, in elements
  static constexpr int NT = KP >= 16 ? KP / 16 : 1;
  static constexpr int KSTEP = KP / 4;          // k-steps of a 16x16x4 product
  static constexpr int TILE_ELEMS = TR * LDST;
  static constexpr int FRAG_ELEMS = KSTEP * NT * kWave;
  static_assert(KP * (int)sizeof(T) >= 16, "row narrower than one vector");
};

// Layout of the FP64 scalar block (k x k products, per-column sums, step
// scalars).  Groups written by one producer are contiguous so that one
// finalize reduces them in a single pass.
template <int KP>
struct SC {
  static constexpr int KK = KP * KP;
  static constexpr int M = 0;                 // X^T X
  static constexpr int GG = M + KK;           // diag G^T G
  static constexpr int GPG = GG + KP;         // diag G_prev^T G
  static constexpr int VPG = GPG + KP;        // diag V_prev^T G
  static constexpr int H = VPG + KP;          // X^T A X
  static constexpr int K = H + KK;            // (AX)^T (AX)
  static constexpr int P = K + KK;            // V^T V
  static constexpr int C = P + KK;            // X^T V
  static constexpr int VG = C + KK;           // diag V^T G
  static constexpr int FD = VG + KP;          // diag V^T A V
  static constexpr int E = FD + KP;           // X^T A V
  static constexpr int F = E + KK;            // V^T A V
  static constexpr int GGP = F + KK;          // diag G_prev^T G_prev
  static constexpr int BETA = GGP + KP;
  static constexpr int ALPHA = BETA + KP;
  static constexpr int COEF = ALPHA + KP;     // 4 * KP: coef[4 i + j] = a_{3-j}
  static constexpr int NROOT = COEF + 4 * KP;
  static constexpr int RELRES = NROOT + KP;
  static constexpr int FVAL = RELRES + 1;
  static constexpr int TOTAL = FVAL + 1;
};

// Device status bits (OR-ed by kernels, mapped to ofm_status on the host).
enum : int { kStNonfinite = 1, kStCholesky = 2, kStNoRoot = 4 };

// Epilogue / pass modes.
enum Mode : int {
  kApply = 0,     // Y = A Z
  kGF1 = 1,       // G = c (AX + X M'), gg, gpg [, vpg] [, H, K]
  kAXF2 = 2,      // store AX, H [, K]
  kAVF1 = 3,      // diag V^T A V
  kAVF2 = 4,      // diag V^T A V, X^T A V, V^T A V
  kGPassF2 = 5,   // G = a AX - b (X H' + AX M'), gg, gpg [, vpg]
  kVPass = 6,     // V = -G + beta V_prev, V^T V, X^T V, diag V^T G
  kUpdate = 7,    // X += alpha V, X^T X
  kGramM = 8,     // X^T X
  kGGP = 9,       // diag G_prev^T G_prev
  kUpdateR = 10,  // X += alpha V, AX += alpha AV, X^T X [, X^T A X]
  kGPassF1 = 11,  // G = c (AX + X M') from a stored AX, gg, gpg [, vpg]
  kGF2 = 12,      // G = a AX - b (X H' + AX M') from the gathered AX, gg, gpg [, vpg] [, H, K]
  kEF = 13,       // X^T A V, V^T A V from a stored A V
  kSF2 = 14,      // S = V^T U, U_i = sum_{j in copy row i} w_ij V_j (upper-triangle copy), in F's slot
  kVPassE = 15    // kVPass and E = (AX)^T V = X^T A V (A symmetric) from a stored A X (k <= 32);
                  // writes [P | C | diag V^T G | 0 (diag V^T A V, unused by f2) | E]
};

struct LaplacianDev {
  int64_t n = 0, nnz = 0;
  int device = 0;
  double normA2 = 0.0;
  double* deg = nullptr;       // [n]
  double* dinv = nullptr;      // [n]
  int32_t* sched = nullptr;    // [n] processing position -> row
  int32_t* sptr = nullptr;     // [n+1] entry offsets by position
  int32_t* tiles = nullptr;    // [ntiles+1] first position of every tile
  int64_t ntiles = 0;
  int tile_rows = 0;           // TR the tile table was built for
  int tile_kind = -1;          // (precision, k) pair the tiles were built for
  void* pk32 = nullptr;        // [nnz] {int col, float w} in position order
  void* pk64 = nullptr;        // [nnz] {int col, int pad, double w}
  int32_t* row_ptr = nullptr;  // [n+1] own copy of the input CSR
  int32_t* col_idx = nullptr;  // [nnz]
  double* w64_csr = nullptr;   // [nnz] w_ij in input CSR order
  bool reorder = true;
  int cold_below = 0;          // columns of rows with fewer entries carry the cold mark
  // upper-triangle copy for the products with A V: of each pair (i, j), (j, i)
  // the entry whose column is later by (degree, id); rows with at least one
  // such entry, by that count, descending, or in the grouped order (nu rows,
  // nnzu entries; none when nu == 0)
  int64_t nu = 0, nnzu = 0;
  int32_t* usched = nullptr;   // [nu] upper position -> row
  int32_t* usptr = nullptr;    // [nu+1]
  void* upk32 = nullptr;       // [nnzu] {int col, float w}
  void* upk64 = nullptr;       // [nnzu] {int col, int pad, double w}
};

// Arguments of the N x k kernels (everything a mode may need).
struct PassArgs {
  int64_t n = 0;
  int k = 0;
  int mode = 0;
  int variant = 0;
  int flags = 0;          // kFlagCheck, kFlagRestart, kFlagFirst
  const void* Z = nullptr;     // SpMM input (X or V); AV for kUpdateR
  void* Y = nullptr;           // SpMM plain output (Y, AX or AV); AX for kUpdateR
  const void* X = nullptr;     // own X rows
  void* Xw = nullptr;          // X written by the update pass
  const void* AX = nullptr;
  void* G = nullptr;           // current direction (written or read)
  const void* Gp = nullptr;    // previous direction
  const void* Vp = nullptr;    // previous search direction
  void* V = nullptr;           // current search direction
  double* sc = nullptr;        // scalar block
  double* partials = nullptr;  // [blocks][nv]
  int nv = 0;
  int nblocks = 0;
  int* status = nullptr;
  // graph (SpMM only)
  const int32_t* sched = nullptr;
  const int32_t* sptr = nullptr;
  const int32_t* tiles = nullptr;
  int64_t ntiles = 0;
  const void* pk = nullptr;
  int cold_below = 0;          // rows with fewer entries are cold (kFlagHC)
  // XCD slots (grouped order): the workgroups b with b % 8 == x walk the tiles
  // [xt[x], xt[x+1]) in chunks of xr * (waves per workgroup) tiles; the grid
  // is then a multiple of 8 workgroups
  int xcd = 0;
  int xr = 1;
  int32_t xt[9] = {};
  // BF16 copies: gather source of the SpMM (null: gather Z itself) and the
  // copies written by the producing passes
  const void* Zg = nullptr;
  void* Xb = nullptr;
  void* Vb = nullptr;
};

// kFlagHC: gathers of rows with the cold mark use the non-temporal policy
// kFlagUpper (kAVF1): the graph is the upper-triangle copy and the pass sums
// V_ic (sum_{j in copy row i} w_ij V_jc) per column; the line search then takes
// diag(V^T A V)_c = -(V^T V)_cc - 2 x that sum
enum : int { kFlagCheck = 1, kFlagRestart = 2, kFlagFirst = 4, kFlagH = 8, kFlagHC = 16,
             kFlagUpper = 32 };

// Batched solves: one launch per pass covers every graph of a width group.
struct BatchGraph {
  int64_t n = 0;
  const int32_t* sched = nullptr;
  const int32_t* sptr = nullptr;
  const int32_t* tiles = nullptr;
  int64_t ntiles = 0;
  const void* pk = nullptr;
  // upper-triangle copy of the Laplacian (upk null: none)
  const int32_t* usched = nullptr;
  const int32_t* usptr = nullptr;
  const int32_t* utiles = nullptr;
  int64_t untiles = 0;
  const void* upk = nullptr;
  void* X = nullptr;
  void* V[2] = {nullptr, nullptr};
  void* G[2] = {nullptr, nullptr};
  void* AX = nullptr;
  void* AV = nullptr;          // A V kept for the recurrence of A X (null without it)
  void* Xb = nullptr;
  void* Vb = nullptr;
  double* sc = nullptr;
  double* partials = nullptr;  // [nblk][nv]
  double* lvl2 = nullptr;      // [workers / kFinChunk][nv] group sums of the partial rows
  int* status = nullptr;
  int* active = nullptr;       // 1 while the graph iterates
  int64_t* done_iter = nullptr;  // iteration whose X met the tolerance (-1: none)
  double* hist = nullptr;      // [kBatchHist] residuals of the last checks (ring)
  int* stalled = nullptr;      // 1 when the residual stopped decreasing
  double normA2 = 0.0;
};
constexpr int kBatchHist = 10;   // checks compared by the stall test
constexpr int kBatchMaxWorkers = 128;  // workgroups per XCD in a batched pass
struct BatchArgs {
  const BatchGraph* graphs = nullptr;
  const int* xlist = nullptr;  // graphs ordered by XCD
  const int* xoff = nullptr;   // [9]: graphs of XCD x are xlist[xoff[x] .. xoff[x+1])
  int workers = 1;             // blocks per XCD; block b is worker b / 8 of XCD b % 8
  int tpw = 4;                 // target tiles per wavefront: a graph uses
                               // min(workers, ceil(tiles / (waves per block * tpw))) workers
  int ngraphs = 0;
  int k = 0;
  int variant = 0;
  int mode = 0;
  int flags = 0;     // kFlagCheck / kFlagRestart / kFlagFirst
  int cur = 0;       // ping-pong slot of the current direction
  int bf16 = 0;      // gather BF16 copies
  double tol = 0.0;
  double freeze_eps = 0.0;
  int64_t t = 0;
  int64_t* tcount = nullptr;   // the group's step counter on the device: read by the
                               // residual, advanced by the line search of every step
  int check_every = 1;
  int nv = 0;
  int off = 0;       // first scalar slot the mode's products go to
  int upper = 0;     // f1: diag(V^T A V) from the upper-triangle copies (graphs that have one)
};
// Persistent form of the lockstep loop (f1 / TriOFM-f1, FP32 without BF16
// copies, two products with A per update, k <= 32): `steps` updates from step
// t0 (slot cur0) of one width group in one cooperative launch.  The BatchArgs
// of each pass carry its mode, flags, nv and off, one copy per ping-pong slot.
enum { kPGF1 = 0, kPGF1C, kPVPass, kPAV, kPUpdate, kPPasses };  // kPGF1C: a checked step
struct BatchPersistArgs {
  BatchArgs pass[kPPasses][2];  // [pass][cur]
  int64_t t0 = 0;
  int cur0 = 0;
  int steps = 0;
  double alpha0 = 0.0;
  unsigned* bar = nullptr;  // [2] zeroed: arrivals, generation
  int* err = nullptr;       // set when a barrier wait timed out
};
// workers per XCD: at most max_workers and what stays resident; the count
// used is returned in *used_workers
hipError_t launch_batch_persist(int k, BatchPersistArgs& p, int max_workers, int* used_workers,
                                hipStream_t s);
hipError_t launch_batch_spmm(int k, BatchArgs& b, hipStream_t s);
hipError_t launch_batch_dense(int k, BatchArgs& b, hipStream_t s);
hipError_t launch_batch_finalize(BatchArgs& b, hipStream_t s);
hipError_t launch_batch_linesearch(int k, BatchArgs& b, double alpha0, int first_fixed,
                                   hipStream_t s);
hipError_t launch_batch_residual(int k, BatchArgs& b, hipStream_t s);
int batch_wpb(int k);

// Launchers (ofm_kernels.hip).  Each returns a hipError_t.
hipError_t launch_spmm(int precision, int k, PassArgs& a, hipStream_t s);
hipError_t launch_dense(int precision, int k, PassArgs& a, hipStream_t s);
// out[v] for v < split, out2[v - split] for v >= split (split = nv: one range)
hipError_t launch_finalize(const double* partials, int nb, int nv, double* out, double* lvl2,
                           hipStream_t s, int split, double* out2);
// advance_h: also H := (X + V D)^T A (X + V D) from X^T A V, V^T A V and the
// step sizes D (the f2 directions then need no stored A X)
// upper_fd = 1: the diag(V^T A V) slot holds the upper-triangle sums of a
// kFlagUpper pass, turned into diag(V^T A V) first; 2: the V^T A V slot holds
// S of a kSF2 pass, turned into V^T A V = -V^T V - S - S^T first
hipError_t launch_linesearch(int k, int variant, int first, double alpha0, int advance_h,
                             int upper_fd, double* sc, int* status, const int* frozen,
                             double freeze_eps, hipStream_t s);
hipError_t launch_select_roots(int tri, int64_t count, const double* coef, double* alpha,
                               int32_t* nroots, hipStream_t s);
hipError_t launch_residual(int k, int variant, double normA2, double* sc, int* status,
                           double tol, int* frozen, hipStream_t s);
hipError_t launch_objective(int k, int variant, double normA2, const double* sc, double* out,
                            hipStream_t s);
int tile_rows(int precision, int k);
int pass_blocks(int precision, int k, int64_t ntiles);
int spmm_wpb(int precision, int k);
int partial_nv(int k, int mode, int flags);
int partial_off(int k, int mode);

// Graph build (ofm_graph.hip)
hipError_t launch_graph_check(int64_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, const double* vals, double* deg,
                              int* flags, hipStream_t s);
hipError_t launch_graph_symcheck(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                 const double* vals, int* flags, hipStream_t s);
hipError_t launch_graph_weights(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                const double* vals, const double* deg, double* dinv,
                                double* w64, double* normA2_parts, hipStream_t s);
hipError_t launch_graph_pack(int64_t n, const int32_t* sched, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* w64, const int32_t* sptr,
                             void* pk32, void* pk64, int cold_below, hipStream_t s);
hipError_t launch_graph_upper_count(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                    int32_t* ucnt, int* flags, hipStream_t s);
hipError_t launch_graph_pack_upper(int64_t nu, const int32_t* usched, const int32_t* row_ptr,
                                   const int32_t* col_idx, const double* w64,
                                   const int32_t* usptr, void* pk32, void* pk64, int cold_below,
                                   hipStream_t s);

// Post-processing (ofm_post.hip)
hipError_t launch_convert(int64_t count, int to_fp64, const void* src, void* dst, hipStream_t s);
hipError_t launch_scale(int64_t count, int precision, const double* sp, const void* X, void* Y,
                        hipStream_t s);
hipError_t launch_row_normalize(int64_t n, int k, int precision, const void* X, void* Y,
                                hipStream_t s);
hipError_t launch_kmeans_assign(int64_t n, int dim, int nc, const float* Y, const float* C,
                                int32_t* labels, float* dist2, hipStream_t s);
hipError_t launch_kmeans_centroid_sums(int64_t n, int dim, int nc, const float* Y,
                                       const int32_t* labels, double* part, int nb,
                                       hipStream_t s);
hipError_t launch_kmeans_centroid_final(int dim, int nc, const double* part, int nb,
                                        const float* old_c, float* new_c, hipStream_t s);
hipError_t launch_kmeans_mindist(int64_t n, int dim, const float* Y, const float* centre,
                                 float* d2, int first, double* sums, hipStream_t s);
hipError_t launch_kmeans_pick(int64_t n, const float* d2, double u, const double* sums,
                              int32_t* pick, hipStream_t s);
hipError_t launch_kmeans_copy_centre(int dim, const float* Y, const int32_t* pick,
                                     float* C, int c, hipStream_t s);
hipError_t launch_count_changes(int64_t n, const int32_t* a, const int32_t* b, int* out,
                                hipStream_t s);
hipError_t launch_gather_rows(int64_t nrows, int S, int row_floats, const int32_t* idx,
                              const float* Z, float* Y, hipStream_t s);
int kmeans_blocks(int64_t n, int nv);
int kmeans_pick_chunks(int64_t n);

}  // namespace ofm
