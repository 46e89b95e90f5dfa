// Kernels of the orthogonalization-free iteration on gfx950.
//
// One iteration of Algorithm 2 (Pang & Yang, arXiv 2305.10356) is a short
// sequence of N x k passes, each ending in a deterministic reduction of
// FP64 k x k products:
//   SpMM(X) with a fused epilogue   -> G (f1 variants) or AX (f2 variants)
//   [G pass for the f2 variants]
//   V pass: V = -G + beta V_prev,  V^T V, X^T V, diag V^T G
//   SpMM(V) with a fused epilogue    -> diag V^T A V [, X^T A V, V^T A V]
//   line search (one workgroup, FP64)
//   update: X += V diag(alpha),  X^T X
// Rows are tiled 16 at a time per wavefront; row vectors move as 16-byte
// loads by LPR consecutive lanes; the k x k products run on the matrix
// cores (v_mfma 16x16x4, FP64 for Grams, the working precision for
// X * (k x k)) from LDS-staged tiles.
#include <float.h>
#include <math.h>

#include "ofm_internal.hpp"

namespace ofm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MF;
// Output layout of the 16x16x4 products (inputs: A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k): D[i][j] sits in lane j + 16 (i / 4), register
// i % 4 for the FP32 instruction and in lane j + 16 (i % 4), register i / 4
// for the FP64 one.  out_row gives i for (lane, register).
template <>
struct MF<float> {
  typedef f4 acc_t;
  __device__ static inline int out_row(int lane, int q) { return 4 * (lane >> 4) + q; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MF<double> {
  typedef d4 acc_t;
  __device__ static inline int out_row(int lane, int q) { return 4 * q + (lane >> 4); }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T, int KP>
using GramAcc = d4[Geo<T, KP>::NT][Geo<T, KP>::NT];
template <typename T, int KP>
using ColAcc = double[3][Geo<T, KP>::VECN];

__device__ inline d4 mma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename T>
struct V16 {
  T v[16 / sizeof(T)];
};

template <typename T>
__device__ inline V16<T> ld16(const T* p) {
  V16<T> r;
  *reinterpret_cast<uint4*>(&r) = *reinterpret_cast<const uint4*>(p);
  return r;
}
template <typename T>
__device__ inline void st16(T* p, const V16<T>& r) {
  *reinterpret_cast<uint4*>(p) = *reinterpret_cast<const uint4*>(&r);
}
// a row part read once in a pass: with NT the load carries the non-temporal
// hint
template <bool NT, typename T>
__device__ inline V16<T> ld16_in(const T* p) {
  if constexpr (NT) {
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    const u4v v = __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p));
    V16<T> r;
    __builtin_memcpy(&r, &v, 16);
    return r;
  } else {
    return ld16(p);
  }
}
// a streamed output row part: with NT the store carries the non-temporal
// hint (used with the hot/cold gathers, so that outputs written once do not
// take cache room from the rows gathered often)
template <bool NT, typename T>
__device__ inline void st16_out(T* p, const V16<T>& r) {
  if constexpr (NT) {
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    u4v v;
    __builtin_memcpy(&v, &r, 16);
    __builtin_nontemporal_store(v, reinterpret_cast<u4v*>(p));
  } else {
    st16(p, r);
  }
}

struct __align__(8) Ent32 {
  int col;
  float w;
};
struct __align__(16) Ent64 {
  int col;
  int pad;
  double w;
};
template <typename T>
struct EntT;
template <>
struct EntT<float> {
  typedef Ent32 type;
};
template <>
struct EntT<double> {
  typedef Ent64 type;
};

// waves per block: keep the dynamic LDS of a block under kLdsBlockCap (a
// workgroup may hold up to 160 KB on this chip).  90 KB gives four waves per
// workgroup to FP32 k = 64 and FP64 k = 32 (two below 67 KB): the FP32 k = 64
// SpMM of X is then held to 2 instead of 1.5 waves per SIMD by its registers
// rather than by its LDS (2.05 -> 1.85 ms on a 2M-node graph; the dense passes
// lose 15-36 us), FP64 k = 32 is unchanged (215 vs 215 iterations/s).
#ifndef OFM_LDS_BLOCK_CAP
#define OFM_LDS_BLOCK_CAP (90 * 1024)
#endif
constexpr int kLdsBlockCap = OFM_LDS_BLOCK_CAP;
template <typename T, int KP>
struct Cfg {
  static constexpr int TB = Geo<T, KP>::TILE_ELEMS * (int)sizeof(T);
  static constexpr int FB = Geo<T, KP>::FRAG_ELEMS * (int)sizeof(T);
  static constexpr int per_wave = 3 * TB + Geo<T, KP>::TR * 4;
  static constexpr int WPB = (2 * FB + 4 * per_wave <= kLdsBlockCap)   ? 4
                             : (2 * FB + 2 * per_wave <= kLdsBlockCap) ? 2
                                                                       : 1;
};

constexpr int nbuf_of(int mode) {
  return (mode == kGF1 || mode == kGF2 || mode == kEF) ? 3
         : (mode == kAXF2 || mode == kSF2) ? 2
         : mode == kAVF2 ? 3
         : (mode == kGPassF2 || mode == kGPassF1) ? 3
         : mode == kVPassE ? 3
         : (mode == kVPass || mode == kUpdateR) ? 2
         : (mode == kUpdate || mode == kGramM) ? 1
                                                : 0;
}
constexpr int nfrag_of(int mode) {
  return (mode == kGF1 || mode == kGPassF1) ? 1 : (mode == kGPassF2 || mode == kGF2) ? 2 : 0;
}
constexpr int nvec_of(int mode) {
  return (mode == kGF1 || mode == kGF2 || mode == kGPassF2 || mode == kGPassF1) ? 3
         : (mode == kVPass || mode == kVPassE || mode == kAVF1 || mode == kAVF2 || mode == kGGP) ? 1
                                                                               : 0;
}

template <typename T, int KP, int MODE>
struct Smem {
  using G = Geo<T, KP>;
  static constexpr int WPB = Cfg<T, KP>::WPB;
  static constexpr int NB = nbuf_of(MODE);
  static constexpr int frag_bytes = nfrag_of(MODE) * G::FRAG_ELEMS * (int)sizeof(T);
  static constexpr int wave_bytes = NB * G::TILE_ELEMS * (int)sizeof(T) + G::TR * 4;
  static constexpr int main_bytes = frag_bytes + WPB * wave_bytes;
  static constexpr int red_bytes = (KP * KP > 3 * KP ? KP * KP : 3 * KP) * 8;
  static constexpr int bytes = main_bytes > red_bytes ? main_bytes : red_bytes;
};

// ---------------------------------------------------------------------------
// partial-row layout of every mode (relative to the first SC slot it fills)
// ---------------------------------------------------------------------------

template <int KP>
__host__ __device__ inline int mode_nv(int mode, int flags) {
  const int KK = KP * KP;
  switch (mode) {
    case kGF1:
    case kGF2: return 3 * KP + ((flags & kFlagCheck) ? 2 * KK : 0);
    case kAXF2: return KK + ((flags & kFlagCheck) ? KK : 0);
    case kAVF1: return KP;
    case kAVF2: return KP + 2 * KK;
    case kGPassF2:
    case kGPassF1: return 3 * KP;
    case kVPass: return 2 * KK + KP;
    case kVPassE: return 3 * KK + 2 * KP;
    case kSF2: return KK;
    case kUpdateR: return KK + ((flags & kFlagH) ? KK : 0);
    case kUpdate:
    case kGramM: return KK;
    case kGGP: return KP;
    case kEF: return 2 * KK;
    default: return 0;
  }
}
template <int KP>
__host__ __device__ inline int mode_off(int mode) {
  switch (mode) {
    case kGF1:
    case kGF2:
    case kGPassF2:
    case kGPassF1: return SC<KP>::GG;
    case kAXF2: return SC<KP>::H;
    case kAVF1:
    case kAVF2: return SC<KP>::FD;
    case kVPass:
    case kVPassE: return SC<KP>::P;
    case kUpdate:
    case kUpdateR:
    case kGramM: return SC<KP>::M;
    case kGGP: return SC<KP>::GGP;
    case kEF: return SC<KP>::E;
    case kSF2: return SC<KP>::F;
    default: return 0;
  }
}

// ---------------------------------------------------------------------------
// wavefront building blocks
// ---------------------------------------------------------------------------

// FP32 -> BF16 with round to nearest even (NaN stays a quiet NaN)
__device__ inline uint32_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// store the VECN (= 4) FP32 values of a lane as BF16 at row r, lane part j
template <int KP>
__device__ inline void st_bf16(void* base, size_t r, int j, const V16<float>& x) {
  uint2 u;
  u.x = f32_to_bf16(x.v[0]) | (f32_to_bf16(x.v[1]) << 16);
  u.y = f32_to_bf16(x.v[2]) | (f32_to_bf16(x.v[3]) << 16);
  *reinterpret_cast<uint2*>(static_cast<uint16_t*>(base) + r * KP + j * 4) = u;
}

// lane part j of gathered row c: 16 bytes of T, or 4 BF16 values widened
template <typename T, int KP, bool BF>
__device__ inline V16<T> load_row_part(const void* Z, int c, int j) {
  using G = Geo<T, KP>;
  if constexpr (!BF) {
    return ld16(static_cast<const T*>(Z) + (size_t)c * KP + j * G::VECN);
  } else {
    static_assert(sizeof(T) == 4, "BF16 gathers feed FP32 arithmetic");
    const uint2 u =
        *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(Z) + (size_t)c * KP + j * 4);
    V16<T> r;
    r.v[0] = __uint_as_float(u.x << 16);
    r.v[1] = __uint_as_float(u.x & 0xffff0000u);
    r.v[2] = __uint_as_float(u.y << 16);
    r.v[3] = __uint_as_float(u.y & 0xffff0000u);
    return r;
  }
}

// lane part j of gathered row c through a buffer load whose cache policy is
// an immediate: AUX = 2 is the non-temporal policy, 0 the default.  The byte
// offset fits in 31 bits (the hot/cold path is taken only for such blocks).
template <typename T, int KP, int AUX>
__device__ inline V16<T> load_row_buf(__amdgpu_buffer_rsrc_t r, int c, int j) {
  using G = Geo<T, KP>;
  const int off = (c * KP + j * G::VECN) * (int)sizeof(T);
  const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, AUX);
  V16<T> v;
  __builtin_memcpy(&v, &u, 16);
  return v;
}

// buffer resource over the N x KP block Z (raw, bounds-checked by size)
template <typename T, int KP>
__device__ inline __amdgpu_buffer_rsrc_t block_rsrc(const void* Z, int64_t n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(Z), (short)0,
                                           (int)(n * KP * (int64_t)sizeof(T)), 0x00020000);
}

// Sum of S_ij-weighted rows Z_j over entries [e_first, end) taken in chunks;
// the LPR lanes of a group share every entry through lane shuffles.  The
// sign bit of a packed column index is the cold mark: masked off, or with HC
// it selects the non-temporal policy for that row's gather.
template <typename T, int KP, bool BF = false, bool HC = false>
__device__ inline void gather_rows(const typename EntT<T>::type* __restrict__ pk,
                                   const void* __restrict__ Z, int e_first, int end, int cstride,
                                   int gbase, int j, V16<T>& acc,
                                   __amdgpu_buffer_rsrc_t zr = __amdgpu_buffer_rsrc_t()) {
  using G = Geo<T, KP>;
  constexpr int CH = G::LPR >= kGatherChunk ? G::LPR : kGatherChunk;
  constexpr int PER = CH / G::LPR;
  for (int e0 = e_first; e0 < end; e0 += cstride) {
    int col[PER];
    T w[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = e0 + u * G::LPR + j;
      if (e < end) {
        const auto en = pk[e];
        col[u] = en.col;
        w[u] = en.w;
      } else {
        col[u] = 0;
        w[u] = T(0);
      }
    }
    V16<T> z[CH];
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const int src = gbase + (s % G::LPR);
      const int cm = __shfl(col[s / G::LPR], src);
      const int c = cm & 0x7fffffff;
      if (e0 + s < end) {
        if constexpr (HC) {
          if (cm < 0) z[s] = load_row_buf<T, KP, 2>(zr, c, j);
          else z[s] = load_row_buf<T, KP, 0>(zr, c, j);
        } else {
          z[s] = load_row_part<T, KP, BF>(Z, c, j);
        }
      } else {
#pragma unroll
        for (int q = 0; q < G::VECN; ++q) z[s].v[q] = T(0);
      }
    }
#pragma unroll
    for (int s = 0; s < CH; ++s) {
      const int src = gbase + (s % G::LPR);
      const T ww = __shfl(w[s / G::LPR], src);
#pragma unroll
      for (int q = 0; q < G::VECN; ++q) acc.v[q] = fma(ww, z[s].v[q], acc.v[q]);
    }
  }
}

template <typename T, int KP>
__device__ inline void tile_store_vec(T* tile, int r, int j, const V16<T>& x) {
  using G = Geo<T, KP>;
#pragma unroll
  for (int q = 0; q < G::VECN; ++q) tile[r * G::LDST + j * G::VECN + q] = x.v[q];
}
template <typename T, int KP>
__device__ inline V16<T> tile_load_vec(const T* tile, int r, int j) {
  using G = Geo<T, KP>;
  V16<T> x;
#pragma unroll
  for (int q = 0; q < G::VECN; ++q) x.v[q] = tile[r * G::LDST + j * G::VECN + q];
  return x;
}
template <typename T, int KP>
__device__ inline void tile_zero_rows(T* tile, int from, int lane) {
  using G = Geo<T, KP>;
  for (int e = from * G::LDST + lane; e < G::TR * G::LDST; e += kWave) tile[e] = T(0);
}

// B operand fragments of a k x k matrix (FP64 source) for X * B:
// frag[(s*NT + tj)*64 + l] = B[4s + l/16][16 tj + l%16]; tri keeps the upper
// triangle (including the diagonal) only.
template <typename T, int KP>
__device__ inline void load_frags(T* frag, const double* B, bool tri) {
  using G = Geo<T, KP>;
  for (int e = threadIdx.x; e < G::FRAG_ELEMS; e += blockDim.x) {
    const int l = e & 63;
    const int st = e >> 6;
    const int tj = st % G::NT;
    const int s = st / G::NT;
    const int row = 4 * s + l / 16;
    const int col = 16 * tj + (l & 15);
    double v = 0.0;
    if (col < KP && (!tri || row <= col)) v = B[row * KP + col];
    frag[e] = (T)v;
  }
}

// out tile (C layout -> LDS) += In(16-row sub-tile) * B for every sub-tile.
template <typename T, int KP>
__device__ inline void tile_times_matrix(const T* in, const T* frag, T* out, int lane,
                                         bool accumulate_from_out) {
  using G = Geo<T, KP>;
  using acc_t = typename MF<T>::acc_t;
#pragma unroll
  for (int sub = 0; sub < G::NSUB; ++sub) {
    acc_t acc[G::NT];
#pragma unroll
    for (int tj = 0; tj < G::NT; ++tj) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = sub * 16 + MF<T>::out_row(lane, q);
        const int c = 16 * tj + (lane & 15);
        acc[tj][q] = (accumulate_from_out && c < KP) ? out[r * G::LDST + c] : T(0);
      }
    }
#pragma unroll
    for (int s = 0; s < G::KSTEP; ++s) {
      const T av = in[(sub * 16 + (lane & 15)) * G::LDST + 4 * s + (lane >> 4)];
#pragma unroll
      for (int tj = 0; tj < G::NT; ++tj)
        acc[tj] = MF<T>::mma(av, frag[(s * G::NT + tj) * 64 + lane], acc[tj]);
    }
#pragma unroll
    for (int tj = 0; tj < G::NT; ++tj) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = sub * 16 + MF<T>::out_row(lane, q);
        const int c = 16 * tj + (lane & 15);
        if (c < KP) out[r * G::LDST + c] = acc[tj][q];
      }
    }
  }
}

// FP64 Gram accumulation acc[ti][tj] += P^T Q over the TR rows of two tiles.
template <typename T, int KP, bool SYM>
__device__ inline void tile_gram(const T* Pt, const T* Qt, GramAcc<T, KP>& acc,
                                 int lane) {
  using G = Geo<T, KP>;
  const int f = lane & 15;
#pragma unroll
  for (int sub = 0; sub < G::NSUB; ++sub) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int r = sub * 16 + 4 * s + (lane >> 4);
      double a[G::NT], b[G::NT];
#pragma unroll
      for (int t = 0; t < G::NT; ++t) {
        const int c = 16 * t + f;
        a[t] = (c < KP) ? (double)Pt[r * G::LDST + c] : 0.0;
        b[t] = (c < KP) ? (double)Qt[r * G::LDST + c] : 0.0;
      }
#pragma unroll
      for (int ti = 0; ti < G::NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < G::NT; ++tj)
          if (!SYM || tj >= ti) acc[ti][tj] = mma64(a[ti], b[tj], acc[ti][tj]);
    }
  }
}

// k x k products of a dense pass with the output tiles dealt to the waves of
// the workgroup (used where one wave cannot hold every FP64 accumulator at a
// useful occupancy: FP32 k = 64, and the FP32 k = 32 V pass with X^T A V).
// The WPB waves stage their row tiles in LDS side by side; product p of the
// pass's list -- group 0's 16 x 16 tiles, then group 1's, then group 2's, a
// symmetric group listing its upper triangle -- belongs to wave p % WPB, which
// sums it over the rows of every staged tile.  Group g multiplies staged tile
// sa_g (rows of the output) by staged tile sb_g (columns of the output).  At
// most NG groups, the first of which may be symmetric.
template <typename T, int KP, int WPB, int NG = 2>
struct SplitGram {
  using G = Geo<T, KP>;
  static constexpr int NT = G::NT;
  static constexpr int PER = (NT * (NT + 1) / 2 + (NG - 1) * NT * NT + WPB - 1) / WPB;
  d4 acc[PER];
  // LDS element offsets of the operands within a staging area (wave-uniform:
  // the lane's own row and column are added when reading)
  int offa[PER], offb[PER];
  int wv = 0, nprod = 0, n0 = 0, n1 = 0;
  bool sym0 = false, sym1 = false;

  // group g and output tile (i, jj) of product p
  __device__ void locate(int p, int& g, int& i, int& jj) const {
    g = p < n0 ? 0 : p < n0 + n1 ? 1 : 2;
    int r = g == 0 ? p : g == 1 ? p - n0 : p - n0 - n1;
    const bool sym = g == 0 ? sym0 : g == 1 ? sym1 : false;
    i = 0;
    if (sym) {
      while (r >= NT - i) {
        r -= NT - i;
        ++i;
      }
      jj = i + r;
    } else {
      i = r / NT;
      jj = r % NT;
    }
  }

  __device__ void setup(int wave, int lane, int sa0, int sb0, bool s0, int sa1, int sb1,
                        bool s1, int ngroups, int sa2 = 0, int sb2 = 0) {
    wv = wave;
    sym0 = s0;
    sym1 = s1;
    n0 = s0 ? NT * (NT + 1) / 2 : NT * NT;
    n1 = ngroups > 1 ? (s1 ? NT * (NT + 1) / 2 : NT * NT) : 0;
    const int n2 = ngroups > 2 ? NT * NT : 0;  // a third group is a full product
    nprod = n0 + n1 + n2;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      acc[q] = d4{0.0, 0.0, 0.0, 0.0};
      const int p = q * WPB + wave;
      int g = 0, i = 0, jj = 0;
      if (p < nprod) locate(p, g, i, jj);
      const int sa = g == 0 ? sa0 : g == 1 ? sa1 : sa2;
      const int sb = g == 0 ? sb0 : g == 1 ? sb1 : sb2;
      offa[q] = __builtin_amdgcn_readfirstlane(sa * G::TILE_ELEMS + 16 * i);
      offb[q] = __builtin_amdgcn_readfirstlane(sb * G::TILE_ELEMS + 16 * jj);
    }
  }
  // a wave that holds no products (it still takes part in out's barriers)
  __device__ void none() { nprod = 0; }

  // every staged tile of the workgroup (waves' areas wave_elems apart), in
  // steps of 4 rows.  FREE: a slot this wave does not own is multiplied too
  // (from valid offsets, never written out), so that no branch separates the
  // matrix instructions and the LDS reads of later products overlap them
  // (vpass_ws_kernel at 2M rows: 591 us with a branch per product, 565 us
  // without; 546 us once the offsets were also wave-uniform).  The other
  // passes keep the branch, with the register use their occupancy was set by.
  template <bool FREE = false>
  __device__ void accumulate(const T* stage0, int wave_elems, int lane) {
    const T* lb = stage0 + (lane >> 4) * G::LDST + (lane & 15);
    for (int w = 0; w < WPB; ++w) {
#pragma unroll
      for (int s4 = 0; s4 < 4 * G::NSUB; ++s4) {
        const T* tb = lb + w * wave_elems + 4 * s4 * G::LDST;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          if (q * WPB >= nprod || (!FREE && q * WPB + wv >= nprod)) continue;
          const double x = (double)tb[offa[q]];
          const double y = (double)tb[offb[q]];
          acc[q] = mma64(x, y, acc[q]);
        }
      }
    }
  }

  // group g's products into red (KP x KP, row-major; a symmetric group also
  // fills the lower triangle), then the block copies them to prow[off ..]
  __device__ void out(int g, bool sym, double* red, double* prow, int off, int lane) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int p = q * WPB + wv;
      if (p >= nprod) continue;
      int gq, ti, tj;
      locate(p, gq, ti, tj);
      if (gq != g) continue;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int ra = 16 * ti + MF<double>::out_row(lane, qq);
        const int cb = 16 * tj + (lane & 15);
        red[ra * KP + cb] = acc[q][qq];
        if (sym && tj > ti) red[cb * KP + ra] = acc[q][qq];
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) prow[off + e] = red[e];
    __syncthreads();
  }
};

// passes whose products are dealt to the waves (FP32 k = 64; the FP32 V
// passes at k = 32, which also prefetch)
template <typename T, int KP, int MODE>
constexpr bool split_gram_mode() {
  return sizeof(T) == 4 &&
         ((KP == 64 && (MODE == kVPass || MODE == kUpdate || MODE == kGramM ||
                        MODE == kUpdateR || MODE == kEF)) ||
          (KP == 32 && (MODE == kVPassE || MODE == kVPass)));
}

template <typename T, int KP>
__device__ inline void zero_gram(GramAcc<T, KP>& acc) {
  using G = Geo<T, KP>;
#pragma unroll
  for (int ti = 0; ti < G::NT; ++ti)
#pragma unroll
    for (int tj = 0; tj < G::NT; ++tj) acc[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
}

// Deterministic block reduction of a Gram (waves in order) into LDS red,
// then the block writes it to its partial row at offset off.
template <typename T, int KP, bool SYM>
__device__ inline void block_gram_out(GramAcc<T, KP>& acc, double* red,
                                      double* prow, int off, int wave, int lane, int nwaves) {
  using G = Geo<T, KP>;
  for (int w = 0; w < nwaves; ++w) {
    if (wave == w) {
#pragma unroll
      for (int ti = 0; ti < G::NT; ++ti)
#pragma unroll
        for (int tj = 0; tj < G::NT; ++tj) {
          if (SYM && tj < ti) continue;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int ra = 16 * ti + MF<double>::out_row(lane, q);
            const int cb = 16 * tj + (lane & 15);
            if (ra < KP && cb < KP) {
              const double v = acc[ti][tj][q];
              if (w == 0) red[ra * KP + cb] = v;
              else red[ra * KP + cb] += v;
              if (SYM && tj > ti) {
                if (w == 0) red[cb * KP + ra] = v;
                else red[cb * KP + ra] += v;
              }
            }
          }
        }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < KP * KP; e += blockDim.x) prow[off + e] = red[e];
  __syncthreads();
}

// per-column sums held in row layout (lane j of every group holds columns
// j*VECN..): reduce over the groups of the wave, then over the waves.
template <typename T, int KP, int NV>
__device__ inline void block_vec_out(ColAcc<T, KP>& cacc,
                                     double* red, double* prow, int off, int wave, int lane,
                                     int nwaves) {
  using G = Geo<T, KP>;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int q = 0; q < G::VECN; ++q) {
      double x = cacc[v][q];
#pragma unroll
      for (int o = G::LPR; o < kWave; o <<= 1) x += __shfl_xor(x, o);
      cacc[v][q] = x;
    }
  const int j = lane % G::LPR;
  for (int w = 0; w < nwaves; ++w) {
    if (wave == w && lane < G::LPR) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int q = 0; q < G::VECN; ++q) {
          const int c = v * KP + j * G::VECN + q;
          if (w == 0) red[c] = cacc[v][q];
          else red[c] += cacc[v][q];
        }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < NV * KP; e += blockDim.x) prow[off + e] = red[e];
  __syncthreads();
}

template <typename T>
__device__ inline bool all_finite(T x) {
  return isfinite((double)x);
}

// ---------------------------------------------------------------------------
// SpMM with fused epilogues:  A Z = -Z - D^{-1/2} S D^{-1/2} Z
// ---------------------------------------------------------------------------

// One pass over the tiles brank, brank + nblk, ... of a graph (a grid of its
// own, or a share of a batched launch); writes the block's partial row brank.
template <typename T, int KP, int MODE, bool CHECK, bool BF, bool HC = false>
__device__ __forceinline__ void spmm_body(const PassArgs& a, int brank, int nblk,
                                          unsigned char* smem) {
  using G = Geo<T, KP>;
  using SM = Smem<T, KP, MODE>;
  constexpr int WPB = SM::WPB;
  constexpr int NV = nvec_of(MODE);
  T* frag = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  unsigned char* wbase = smem + SM::frag_bytes + wave * SM::wave_bytes;
  T* tA = reinterpret_cast<T*>(wbase);                                   // A Z rows
  T* tZ = tA + G::TILE_ELEMS;                                            // own Z rows
  T* tD = tZ + G::TILE_ELEMS;                                            // third tile
  int* trow = reinterpret_cast<int*>(wbase + SM::NB * G::TILE_ELEMS * sizeof(T));

  constexpr bool check = CHECK;
  const bool restart = (a.flags & kFlagRestart) != 0;
  // upper-triangle pass: V_i times its sum over the row's entries in the copy
  const bool upper = MODE == kAVF1 && (a.flags & kFlagUpper) != 0;
  const T* __restrict__ Z = static_cast<const T*>(a.Z);
  const auto* __restrict__ pk = static_cast<const typename EntT<T>::type*>(a.pk);
  __amdgpu_buffer_rsrc_t zr = __amdgpu_buffer_rsrc_t();
  if constexpr (HC) zr = block_rsrc<T, KP>(a.Z, a.n);
  const int g = lane / G::LPR;
  const int j = lane % G::LPR;
  const double* sc = a.sc;

  T cf = T(1), ca = T(0), cb = T(0);
  if (MODE == kGF1) {
    load_frags<T, KP>(frag, sc + SC<KP>::M, a.variant == OFM_TRI_F1);
    cf = (a.variant == OFM_F1) ? T(4) : T(1);
    __syncthreads();
  } else if (MODE == kGF2) {
    // the f2 directions with H of the current iterate from the scalar block
    const bool tri = a.variant == OFM_TRI_F2;
    load_frags<T, KP>(frag, sc + SC<KP>::H, tri);                  // H'
    load_frags<T, KP>(frag + G::FRAG_ELEMS, sc + SC<KP>::M, tri);  // M'
    ca = tri ? T(2) : T(4);
    cb = tri ? T(1) : T(2);
    __syncthreads();
  }

  double cacc[3][G::VECN];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < G::VECN; ++q) cacc[v][q] = 0.0;
  d4 gA[G::NT][G::NT], gB[G::NT][G::NT];
  zero_gram<T, KP>(gA);
  zero_gram<T, KP>(gB);

  // tiles of this wave: chunks of `span` consecutive tiles, chunk c0, c0 +
  // cstride, ...; each wave takes every WPB-th tile of a chunk.  Tile indices
  // fit in 32 bits (fewer than n / 16 + nnz / kHeavyDeg tiles); the wave index
  // is made wave-uniform so that the loop lives in scalar registers.
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  int c0 = brank * WPB, tend = (int)a.ntiles, cstride = nblk * WPB, span = WPB;
  if (a.xcd) {
    // grouped order: workgroup b runs on XCD b % 8 and walks that XCD's slot
    // in chunks of xr * WPB tiles
    const int x = brank & 7;
    span = WPB * a.xr;
    c0 = a.xt[x] + (brank >> 3) * span;
    tend = a.xt[x + 1];
    cstride = (nblk >> 3) * span;
  }
  for (; c0 < tend; c0 += cstride)
  for (int t = c0 + wv, cend = c0 + span < tend ? c0 + span : tend; t < cend; t += WPB) {
    const int tinfo = a.tiles[t];
    const int start = tinfo & 0x7fffffff;
    const bool heavy = tinfo < 0;
    const int cnt = (a.tiles[t + 1] & 0x7fffffff) - start;

    if (!heavy) {
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        if (gi < cnt) {
          const int p = start + gi;
          const int beg = a.sptr[p], end = a.sptr[p + 1];
          const int row = a.sched[p];
          V16<T> acc;
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) acc.v[q] = T(0);
          gather_rows<T, KP, BF, HC>(pk, BF ? a.Zg : a.Z, beg, end,
                                     G::LPR >= kGatherChunk ? G::LPR : kGatherChunk, g * G::LPR,
                                     j, acc, zr);
          const V16<T> z = (HC && end - beg < a.cold_below)
                                ? ld16_in<HC>(Z + (size_t)row * KP + j * G::VECN)
                                : ld16(Z + (size_t)row * KP + j * G::VECN);
          if (upper) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)z.v[q] * (double)acc.v[q];
            continue;
          }
          if (MODE != kSF2) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) acc.v[q] = -z.v[q] - acc.v[q];
          }
          if (j == 0) trow[gi] = row;
          if (MODE == kApply || MODE == kAXF2 || (MODE == kGF2 && a.Y)) {
            st16_out<HC>(static_cast<T*>(a.Y) + (size_t)row * KP + j * G::VECN, acc);
          }
          if (MODE == kAVF1 || MODE == kAVF2) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)z.v[q] * (double)acc.v[q];
            if (a.Y) st16_out<HC>(static_cast<T*>(a.Y) + (size_t)row * KP + j * G::VECN, acc);
          }
          if (SM::NB > 0) {
            tile_store_vec<T, KP>(tA, gi, j, acc);
            tile_store_vec<T, KP>(tZ, gi, j, z);
          }
        }
      }
    } else {
      for (int gi = 0; gi < cnt; ++gi) {
        const int p = start + gi;
        const int beg = a.sptr[p], end = a.sptr[p + 1];
        const int row = a.sched[p];
        constexpr int CH = G::LPR >= kGatherChunk ? G::LPR : kGatherChunk;
        V16<T> acc;
#pragma unroll
        for (int q = 0; q < G::VECN; ++q) acc.v[q] = T(0);
        gather_rows<T, KP, BF, HC>(pk, BF ? a.Zg : a.Z, beg + g * CH, end, G::RPW * CH,
                                   g * G::LPR, j, acc, zr);
#pragma unroll
        for (int q = 0; q < G::VECN; ++q) {
#pragma unroll
          for (int o = G::LPR; o < kWave; o <<= 1) acc.v[q] += __shfl_xor(acc.v[q], o);
        }
        if (g == 0) {
          const V16<T> z = (HC && end - beg < a.cold_below)
                                ? ld16_in<HC>(Z + (size_t)row * KP + j * G::VECN)
                                : ld16(Z + (size_t)row * KP + j * G::VECN);
          if (upper) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)z.v[q] * (double)acc.v[q];
            continue;
          }
          if (MODE != kSF2) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) acc.v[q] = -z.v[q] - acc.v[q];
          }
          if (j == 0) trow[gi] = row;
          if (MODE == kApply || MODE == kAXF2 || (MODE == kGF2 && a.Y)) {
            st16_out<HC>(static_cast<T*>(a.Y) + (size_t)row * KP + j * G::VECN, acc);
          }
          if (MODE == kAVF1 || MODE == kAVF2) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)z.v[q] * (double)acc.v[q];
            if (a.Y) st16_out<HC>(static_cast<T*>(a.Y) + (size_t)row * KP + j * G::VECN, acc);
          }
          if (SM::NB > 0) {
            tile_store_vec<T, KP>(tA, gi, j, acc);
            tile_store_vec<T, KP>(tZ, gi, j, z);
          }
        }
      }
    }
    if (SM::NB == 0) continue;
    // rows beyond cnt are zero so that they add nothing to the products
    if (cnt < G::TR) {
      tile_zero_rows<T, KP>(tA, cnt, lane);
      tile_zero_rows<T, KP>(tZ, cnt, lane);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");

    if (MODE == kGF1 || MODE == kGF2) {
      // kGF1: D = X M', G = c (AX + D); kGF2: D = X H' + AX M', G = ca AX - cb D;
      // per-column sums of G*G, G_prev*G, V_prev*G
      tile_times_matrix<T, KP>(tZ, frag, tD, lane, false);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      if (MODE == kGF2) {
        tile_times_matrix<T, KP>(tA, frag + G::FRAG_ELEMS, tD, lane, true);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      }
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        if (gi < cnt) {
          const int row = trow[gi];
          const V16<T> ax = tile_load_vec<T, KP>(tA, gi, j);
          const V16<T> d = tile_load_vec<T, KP>(tD, gi, j);
          V16<T> gv;
          if (MODE == kGF1) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) gv.v[q] = cf * (ax.v[q] + d.v[q]);
          } else {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) gv.v[q] = ca * ax.v[q] - cb * d.v[q];
          }
          const size_t off = (size_t)row * KP + j * G::VECN;
          st16_out<HC>(static_cast<T*>(a.G) + off, gv);
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)gv.v[q] * (double)gv.v[q];
          if (a.Gp) {
            const V16<T> gp = ld16_in<HC>(static_cast<const T*>(a.Gp) + off);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[1][q] += (double)gp.v[q] * (double)gv.v[q];
          }
          if (restart && a.Vp) {
            const V16<T> vp = ld16(static_cast<const T*>(a.Vp) + off);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[2][q] += (double)vp.v[q] * (double)gv.v[q];
          }
        }
      }
      if (check) {
        tile_gram<T, KP, false>(tZ, tA, gA, lane);  // H = X^T (AX)
        tile_gram<T, KP, true>(tA, tA, gB, lane);   // K = (AX)^T (AX)
      }
    } else if (MODE == kAXF2) {
      tile_gram<T, KP, false>(tZ, tA, gA, lane);
      if (check) tile_gram<T, KP, true>(tA, tA, gB, lane);
    } else if (MODE == kSF2) {
      tile_gram<T, KP, false>(tZ, tA, gA, lane);  // S = V^T U
    } else if (MODE == kAVF2) {
      // own X rows of the tile
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        V16<T> x;
        if (gi < cnt) {
          x = ld16(static_cast<const T*>(a.X) + (size_t)trow[gi] * KP + j * G::VECN);
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) x.v[q] = T(0);
        }
        if (gi < G::TR) tile_store_vec<T, KP>(tD, gi, j, x);
      }
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      tile_gram<T, KP, false>(tD, tA, gA, lane);  // E = X^T (AV)
      tile_gram<T, KP, true>(tZ, tA, gB, lane);   // F = V^T (AV)
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }

  // block partial row
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  if (MODE == kApply) return;
  double* prow = a.partials + (size_t)brank * a.nv;
  const int KK = KP * KP;
  if (MODE == kGF1 || MODE == kGF2) {
    block_vec_out<T, KP, 3>(cacc, red, prow, 0, wave, lane, WPB);
    if (check) {
      block_gram_out<T, KP, false>(gA, red, prow, 3 * KP, wave, lane, WPB);
      block_gram_out<T, KP, true>(gB, red, prow, 3 * KP + KK, wave, lane, WPB);
    }
  } else if (MODE == kAXF2) {
    block_gram_out<T, KP, false>(gA, red, prow, 0, wave, lane, WPB);
    if (check) block_gram_out<T, KP, true>(gB, red, prow, KK, wave, lane, WPB);
  } else if (MODE == kAVF1) {
    block_vec_out<T, KP, 1>(cacc, red, prow, 0, wave, lane, WPB);
  } else if (MODE == kSF2) {
    block_gram_out<T, KP, false>(gA, red, prow, 0, wave, lane, WPB);
  } else if (MODE == kAVF2) {
    block_vec_out<T, KP, 1>(cacc, red, prow, 0, wave, lane, WPB);
    block_gram_out<T, KP, false>(gA, red, prow, KP, wave, lane, WPB);
    block_gram_out<T, KP, true>(gB, red, prow, KP + KK, wave, lane, WPB);
  }
}

// ---------------------------------------------------------------------------
// N x k streaming passes
// ---------------------------------------------------------------------------

template <typename T, int KP, int MODE>
__device__ __forceinline__ void dense_body(const PassArgs& a, int brank, int nblk,
                                           unsigned char* smem) {
  using G = Geo<T, KP>;
  using SM = Smem<T, KP, MODE>;
  constexpr int WPB = SM::WPB;
  constexpr int NV = nvec_of(MODE);
  T* frag = reinterpret_cast<T*>(smem);
  T* frag2 = frag + G::FRAG_ELEMS;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  unsigned char* wbase = smem + SM::frag_bytes + wave * SM::wave_bytes;
  T* t0 = reinterpret_cast<T*>(wbase);
  T* t1 = t0 + G::TILE_ELEMS;
  T* t2 = t1 + G::TILE_ELEMS;
  const int g = lane / G::LPR;
  const int j = lane % G::LPR;
  const double* sc = a.sc;
  const bool restart = (a.flags & kFlagRestart) != 0;
  const bool first = (a.flags & kFlagFirst) != 0;
  constexpr bool VP = MODE == kVPass || MODE == kVPassE;
  constexpr bool HASE = MODE == kVPassE;  // the V pass that also forms E

  // per-column scalars of this pass (beta for V, alpha for the update)
  T colscal[G::VECN];
#pragma unroll
  for (int q = 0; q < G::VECN; ++q) colscal[q] = T(0);
  T ca = T(0), cb = T(0);
  if (VP) {
#pragma unroll
    for (int q = 0; q < G::VECN; ++q) {
      const int c = j * G::VECN + q;
      double beta = 0.0;
      if (!first) {
        const double den = sc[SC<KP>::GGP + c];
        const double num = sc[SC<KP>::GG + c] - sc[SC<KP>::GPG + c];
        beta = (den != 0.0) ? num / den : 0.0;
        if (restart && (-sc[SC<KP>::GG + c] + beta * sc[SC<KP>::VPG + c]) >= 0.0) beta = 0.0;
      }
      colscal[q] = (T)beta;
      if (brank == 0 && threadIdx.x < G::LPR) const_cast<double*>(sc)[SC<KP>::BETA + c] = beta;
    }
  } else if (MODE == kUpdate || MODE == kUpdateR) {
#pragma unroll
    for (int q = 0; q < G::VECN; ++q) colscal[q] = (T)sc[SC<KP>::ALPHA + j * G::VECN + q];
  } else if (MODE == kGPassF1) {
    // G = c (AX + X M'): the direction kGF1 forms, with AX read from memory
    const bool tri = a.variant == OFM_TRI_F1;
    load_frags<T, KP>(frag, sc + SC<KP>::M, tri);
    ca = tri ? T(1) : T(4);
    cb = -ca;
    __syncthreads();
  } else if (MODE == kGPassF2) {
    const bool tri = a.variant == OFM_TRI_F2;
    load_frags<T, KP>(frag, sc + SC<KP>::H, tri);   // H'
    load_frags<T, KP>(frag2, sc + SC<KP>::M, tri);  // M'
    ca = tri ? T(2) : T(4);
    cb = tri ? T(1) : T(2);
    __syncthreads();
  }

  double cacc[3][G::VECN];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < G::VECN; ++q) cacc[v][q] = 0.0;
  constexpr bool SPLIT = split_gram_mode<T, KP, MODE>();
  d4 gA[G::NT][G::NT], gB[G::NT][G::NT];  // per-wave products (unused with SPLIT)
  zero_gram<T, KP>(gA);
  zero_gram<T, KP>(gB);
  constexpr int NTE = HASE ? G::NT : 1;
  d4 gE[NTE][NTE];                         // E = (AX)^T V (kVPassE)
#pragma unroll
  for (int ti = 0; ti < NTE; ++ti)
#pragma unroll
    for (int tj = 0; tj < NTE; ++tj) gE[ti][tj] = d4{0.0, 0.0, 0.0, 0.0};
  SplitGram<T, KP, WPB, HASE ? 3 : 2> sg;
  if constexpr (SPLIT) {
    // (source tiles, symmetry) of the product groups: t0 = 0, t1 = 1, t2 = 2
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    if (MODE == kVPass) sg.setup(wv, lane, 0, 0, true, 1, 0, false, 2);      // P = V^T V, C = X^T V
    else if (MODE == kVPassE)                                                 // P, C, E = (AX)^T V
      sg.setup(wv, lane, 0, 0, true, 1, 0, false, 3, 2, 0);
    else if (MODE == kEF) sg.setup(wv, lane, 0, 2, false, 1, 2, true, 2);    // E = X^T AV, F = V^T AV
    else if (MODE == kUpdateR)
      sg.setup(wv, lane, 0, 0, true, 0, 1, false, (a.flags & kFlagH) ? 2 : 1);  // M [, H = X^T AX]
    else sg.setup(wv, lane, 0, 0, true, 0, 0, false, 1);                     // M = X^T X
  }

  const int64_t ntiles = (a.n + G::TR - 1) / G::TR;
  const int64_t stride = (int64_t)nblk * WPB;
  // The FP32 k = 32 V passes (split products) prefetch: each wave issues the
  // global loads of its next tile before the workgroup's products over the
  // staged tiles (a workgroup barrier waits for the LDS only, so the loads
  // stay in flight through the products): at N = 2M the V pass with X^T A V
  // 299 -> 267 us, the plain one 202 (unsplit) -> 194 us.  The loop below then
  // does not run.  At k = 64 the prefetch registers cost the V pass a wave per
  // SIMD and it measured slower (678 -> 753 us).
  constexpr bool PF = SPLIT && VP && KP <= 32;
  if constexpr (PF) {
    V16<T> pg[G::NPASS], px[G::NPASS], pv[G::NPASS], pa[G::NPASS];
    auto fetch = [&](int64_t tbn) {
      const int64_t tn = tbn + wave;
      const int64_t rn = tn * G::TR;
      const int cn = tn >= ntiles ? 0 : (int)((a.n - rn) < G::TR ? (a.n - rn) : G::TR);
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        if (gi < cn) {
          const size_t off = (size_t)(rn + gi) * KP + j * G::VECN;
          pg[pass] = ld16(static_cast<const T*>(a.G) + off);
          px[pass] = ld16(static_cast<const T*>(a.X) + off);
          if (!first) pv[pass] = ld16(static_cast<const T*>(a.Vp) + off);
          if constexpr (HASE) pa[pass] = ld16(static_cast<const T*>(a.AX) + off);
        }
      }
    };
    int64_t tb = (int64_t)brank * WPB;
    if (tb < ntiles) fetch(tb);
    for (; tb < ntiles; tb += stride) {
      const int64_t t = tb + wave;
      const int64_t r0 = t * G::TR;
      const int cnt = t >= ntiles ? 0 : (int)((a.n - r0) < G::TR ? (a.n - r0) : G::TR);
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        const bool ok = gi < cnt;
        const size_t off = (size_t)(r0 + gi) * KP + j * G::VECN;
        V16<T> v, x;
        if (ok) {
          const V16<T> gv = pg[pass];
          x = px[pass];
          if (!first) {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) v.v[q] = fma(colscal[q], pv[pass].v[q], -gv.v[q]);
          } else {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) v.v[q] = -gv.v[q];
          }
          st16(static_cast<T*>(a.V) + off, v);
          if constexpr (sizeof(T) == 4) {
            if (a.Vb) st_bf16<KP>(a.Vb, (size_t)(r0 + gi), j, v);
          }
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)v.v[q] * (double)gv.v[q];
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) v.v[q] = x.v[q] = T(0);
        }
        if (gi < G::TR) {
          tile_store_vec<T, KP>(t0, gi, j, v);
          tile_store_vec<T, KP>(t1, gi, j, x);
        }
        if constexpr (HASE) {
          V16<T> ax;
          if (ok) {
            ax = pa[pass];
          } else {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) ax.v[q] = T(0);
          }
          if (gi < G::TR) tile_store_vec<T, KP>(t2, gi, j, ax);
        }
      }
      if (tb + stride < ntiles) fetch(tb + stride);
      __syncthreads();
      sg.accumulate(reinterpret_cast<const T*>(smem + SM::frag_bytes),
                    SM::wave_bytes / (int)sizeof(T), lane);
      __syncthreads();
    }
  }
  // per wave: tiles brank * WPB + wave + i * stride.  With the split products
  // the WPB waves run the loop together (a wave past the last tile stages
  // zeros) and meet at a barrier before and after the products.
  for (int64_t tb = PF ? ntiles : (int64_t)brank * WPB; tb < ntiles; tb += stride) {
    const int64_t t = tb + wave;
    if (!SPLIT && t >= ntiles) break;
    const int64_t r0 = t * G::TR;
    const int cnt = t >= ntiles ? 0 : (int)((a.n - r0) < G::TR ? (a.n - r0) : G::TR);
#pragma unroll
    for (int pass = 0; pass < G::NPASS; ++pass) {
      const int gi = pass * G::RPW + g;
      const bool ok = gi < cnt;
      const size_t off = (size_t)(r0 + gi) * KP + j * G::VECN;
      if (VP) {
        V16<T> v, gv, x;
        if (ok) {
          gv = ld16(static_cast<const T*>(a.G) + off);
          x = ld16(static_cast<const T*>(a.X) + off);
          if (!first) {
            const V16<T> vp = ld16(static_cast<const T*>(a.Vp) + off);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) v.v[q] = fma(colscal[q], vp.v[q], -gv.v[q]);
          } else {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) v.v[q] = -gv.v[q];
          }
          st16(static_cast<T*>(a.V) + off, v);
          if constexpr (sizeof(T) == 4) {
            if (a.Vb) st_bf16<KP>(a.Vb, (size_t)(r0 + gi), j, v);
          }
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)v.v[q] * (double)gv.v[q];
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) v.v[q] = x.v[q] = T(0);
        }
        if (gi < G::TR) {
          tile_store_vec<T, KP>(t0, gi, j, v);
          tile_store_vec<T, KP>(t1, gi, j, x);
        }
        if constexpr (HASE) {
          V16<T> ax;
          if (ok) {
            ax = ld16(static_cast<const T*>(a.AX) + off);
          } else {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) ax.v[q] = T(0);
          }
          if (gi < G::TR) tile_store_vec<T, KP>(t2, gi, j, ax);
        }
      } else if (MODE == kUpdate || MODE == kGramM) {
        V16<T> x;
        if (ok) {
          x = ld16(static_cast<const T*>(a.X) + off);
          if (MODE == kUpdate) {
            const V16<T> v = ld16(static_cast<const T*>(a.V) + off);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) x.v[q] = fma(colscal[q], v.v[q], x.v[q]);
            st16(static_cast<T*>(a.Xw) + off, x);
          }
          if constexpr (sizeof(T) == 4) {
            if (a.Xb) st_bf16<KP>(a.Xb, (size_t)(r0 + gi), j, x);
          }
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) x.v[q] = T(0);
        }
        if (gi < G::TR) tile_store_vec<T, KP>(t0, gi, j, x);
      } else if (MODE == kEF) {
        V16<T> x, v, av;
        if (ok) {
          x = ld16(static_cast<const T*>(a.X) + off);
          v = ld16(static_cast<const T*>(a.V) + off);
          av = ld16(static_cast<const T*>(a.Z) + off);
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) x.v[q] = v.v[q] = av.v[q] = T(0);
        }
        if (gi < G::TR) {
          tile_store_vec<T, KP>(t0, gi, j, x);
          tile_store_vec<T, KP>(t1, gi, j, v);
          tile_store_vec<T, KP>(t2, gi, j, av);
        }
      } else if (MODE == kUpdateR) {
        V16<T> x, ax;
        if (ok) {
          x = ld16(static_cast<const T*>(a.X) + off);
          ax = ld16(static_cast<const T*>(a.AX) + off);
          const V16<T> v = ld16(static_cast<const T*>(a.V) + off);
          const V16<T> av = ld16(static_cast<const T*>(a.Z) + off);
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) {
            x.v[q] = fma(colscal[q], v.v[q], x.v[q]);
            ax.v[q] = fma(colscal[q], av.v[q], ax.v[q]);
          }
          st16(static_cast<T*>(a.Xw) + off, x);
          st16(static_cast<T*>(a.Y) + off, ax);
          if constexpr (sizeof(T) == 4) {
            if (a.Xb) st_bf16<KP>(a.Xb, (size_t)(r0 + gi), j, x);
          }
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) x.v[q] = ax.v[q] = T(0);
        }
        if (gi < G::TR) {
          tile_store_vec<T, KP>(t0, gi, j, x);
          tile_store_vec<T, KP>(t1, gi, j, ax);
        }
      } else if (MODE == kGGP) {
        if (ok) {
          const V16<T> gp = ld16(static_cast<const T*>(a.Gp) + off);
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)gp.v[q] * (double)gp.v[q];
        }
      } else if (MODE == kGPassF2 || MODE == kGPassF1) {
        V16<T> x, ax;
        if (ok) {
          x = ld16(static_cast<const T*>(a.X) + off);
          ax = ld16(static_cast<const T*>(a.AX) + off);
        } else {
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) x.v[q] = ax.v[q] = T(0);
        }
        if (gi < G::TR) {
          tile_store_vec<T, KP>(t0, gi, j, x);
          tile_store_vec<T, KP>(t1, gi, j, ax);
        }
      }
    }
    if (SM::NB == 0) continue;
    if constexpr (SPLIT) {
      __syncthreads();
      sg.accumulate(reinterpret_cast<const T*>(smem + SM::frag_bytes),
                    SM::wave_bytes / (int)sizeof(T), lane);
      __syncthreads();
      continue;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    if (VP) {
      tile_gram<T, KP, true>(t0, t0, gA, lane);   // P = V^T V
      tile_gram<T, KP, false>(t1, t0, gB, lane);  // C = X^T V
      if constexpr (HASE) tile_gram<T, KP, false>(t2, t0, gE, lane);  // E = (AX)^T V
    } else if (MODE == kUpdate || MODE == kGramM) {
      tile_gram<T, KP, true>(t0, t0, gA, lane);   // M = X^T X
    } else if (MODE == kEF) {
      tile_gram<T, KP, false>(t0, t2, gA, lane);  // E = X^T (AV)
      tile_gram<T, KP, true>(t1, t2, gB, lane);   // F = V^T (AV)
    } else if (MODE == kUpdateR) {
      tile_gram<T, KP, true>(t0, t0, gA, lane);                        // M = X^T X
      if (a.flags & kFlagH) tile_gram<T, KP, false>(t0, t1, gB, lane);  // H = X^T (AX)
    } else if (MODE == kGPassF2 || MODE == kGPassF1) {
      // kGPassF2: D = X H' + AX M'; kGPassF1: D = X M'; then G = ca AX - cb D
      tile_times_matrix<T, KP>(t0, frag, t2, lane, false);
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      if (MODE == kGPassF2) {
        tile_times_matrix<T, KP>(t1, frag2, t2, lane, true);
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      }
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        if (gi < cnt) {
          const size_t off = (size_t)(r0 + gi) * KP + j * G::VECN;
          const V16<T> ax = tile_load_vec<T, KP>(t1, gi, j);
          const V16<T> d = tile_load_vec<T, KP>(t2, gi, j);
          V16<T> gv;
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) gv.v[q] = ca * ax.v[q] - cb * d.v[q];
          st16(static_cast<T*>(a.G) + off, gv);
#pragma unroll
          for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)gv.v[q] * (double)gv.v[q];
          if (a.Gp) {
            const V16<T> gp = ld16(static_cast<const T*>(a.Gp) + off);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[1][q] += (double)gp.v[q] * (double)gv.v[q];
          }
          if (restart && a.Vp) {
            const V16<T> vp = ld16(static_cast<const T*>(a.Vp) + off);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[2][q] += (double)vp.v[q] * (double)gv.v[q];
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  }

  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  double* prow = a.partials + (size_t)brank * a.nv;
  const int KK = KP * KP;
  if constexpr (SPLIT) {
    if (VP) {
      sg.out(0, true, red, prow, 0, lane);
      sg.out(1, false, red, prow, KK, lane);
      block_vec_out<T, KP, 1>(cacc, red, prow, 2 * KK, wave, lane, WPB);
      if (HASE) {
        for (int e = threadIdx.x; e < KP; e += blockDim.x) prow[2 * KK + KP + e] = 0.0;
        sg.out(2, false, red, prow, 2 * KK + 2 * KP, lane);
      }
    } else if (MODE == kEF) {
      sg.out(0, false, red, prow, 0, lane);
      sg.out(1, true, red, prow, KK, lane);
    } else if (MODE == kUpdateR) {
      sg.out(0, true, red, prow, 0, lane);
      if (a.flags & kFlagH) sg.out(1, false, red, prow, KK, lane);
    } else {
      sg.out(0, true, red, prow, 0, lane);
    }
  } else if (VP) {
    block_gram_out<T, KP, true>(gA, red, prow, 0, wave, lane, WPB);
    block_gram_out<T, KP, false>(gB, red, prow, KK, wave, lane, WPB);
    block_vec_out<T, KP, 1>(cacc, red, prow, 2 * KK, wave, lane, WPB);
    if constexpr (HASE) {
      // [.. | diag V^T G | 0 (the diag V^T A V slot, unused by f2) | E]
      for (int e = threadIdx.x; e < KP; e += blockDim.x) prow[2 * KK + KP + e] = 0.0;
      block_gram_out<T, KP, false>(gE, red, prow, 2 * KK + 2 * KP, wave, lane, WPB);
    }
  } else if (MODE == kUpdate || MODE == kGramM) {
    block_gram_out<T, KP, true>(gA, red, prow, 0, wave, lane, WPB);
  } else if (MODE == kUpdateR) {
    block_gram_out<T, KP, true>(gA, red, prow, 0, wave, lane, WPB);
    if (a.flags & kFlagH) block_gram_out<T, KP, false>(gB, red, prow, KK, wave, lane, WPB);
  } else if (MODE == kGGP) {
    block_vec_out<T, KP, 1>(cacc, red, prow, 0, wave, lane, WPB);
  } else if (MODE == kGPassF2 || MODE == kGPassF1) {
    block_vec_out<T, KP, 3>(cacc, red, prow, 0, wave, lane, WPB);
  } else if (MODE == kEF) {
    block_gram_out<T, KP, false>(gA, red, prow, 0, wave, lane, WPB);
    block_gram_out<T, KP, true>(gB, red, prow, KK, wave, lane, WPB);
  }
}

template <typename T, int KP, int MODE, bool CHECK, bool BF, bool HC>
__global__ void __launch_bounds__((Cfg<T, KP>::WPB * 64)) spmm_kernel(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  spmm_body<T, KP, MODE, CHECK, BF, HC>(a, blockIdx.x, gridDim.x, smem);
}

template <typename T, int KP, int MODE>
__global__ void __launch_bounds__((Cfg<T, KP>::WPB * 64)) dense_kernel(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  dense_body<T, KP, MODE>(a, blockIdx.x, gridDim.x, smem);
}

// The FP32 k = 64 V pass with the waves of a workgroup given one job each.
// Waves 0-3 (loaders) stream G, V_prev and X of one 16-row tile each per
// round, form V = -G + V_prev diag(beta), store it and stage the V and X tiles
// in LDS; waves 4-7 hold the FP64 products (V^T V upper triangle and X^T V,
// dealt as in SplitGram) and multiply the tiles staged in the round before.
// The rounds alternate between two staging buffers with one workgroup barrier
// each, so the matrix cores run while the loaders wait for memory, and no
// wave holds both the accumulators and loads in flight.  Partial row:
// [P | C | diag V^T G], as the V pass writes it.
constexpr int kVpwLoaders = 4;
struct VPassWS {
  using G = Geo<float, 64>;
  static constexpr int AREA = 2 * G::TILE_ELEMS;  // V and X tiles of one loader (floats)
  static constexpr int BUF = kVpwLoaders * AREA;  // one round's tiles (floats)
  static constexpr int main_bytes = 2 * BUF * (int)sizeof(float);
  static constexpr int red_bytes = 64 * 64 * 8;
  static constexpr int bytes = main_bytes > red_bytes ? main_bytes : red_bytes;
};

__global__ void __launch_bounds__(2 * kVpwLoaders * 64, 4) vpass_ws_kernel(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int KP = 64;
  using T = float;
  using G = Geo<T, KP>;
  using W = VPassWS;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  const bool loader = wv < kVpwLoaders;
  const int g = lane / G::LPR;
  const int j = lane % G::LPR;
  const double* sc = a.sc;
  const bool restart = (a.flags & kFlagRestart) != 0;
  const bool first = (a.flags & kFlagFirst) != 0;

  T beta_c[G::VECN];
#pragma unroll
  for (int q = 0; q < G::VECN; ++q) {
    const int c = j * G::VECN + q;
    double beta = 0.0;
    if (!first) {
      const double den = sc[SC<KP>::GGP + c];
      const double num = sc[SC<KP>::GG + c] - sc[SC<KP>::GPG + c];
      beta = (den != 0.0) ? num / den : 0.0;
      if (restart && (-sc[SC<KP>::GG + c] + beta * sc[SC<KP>::VPG + c]) >= 0.0) beta = 0.0;
    }
    beta_c[q] = (T)beta;
    if (blockIdx.x == 0 && threadIdx.x < G::LPR) const_cast<double*>(sc)[SC<KP>::BETA + c] = beta;
  }

  double cacc[3][G::VECN];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int q = 0; q < G::VECN; ++q) cacc[v][q] = 0.0;
  SplitGram<T, KP, kVpwLoaders, 2> sg;
  if (loader) {
    sg.none();
  } else {
    sg.setup(wv - kVpwLoaders, lane, 0, 0, true, 1, 0, false, 2);  // P = V^T V, C = X^T V
  }

  const int64_t ntiles = (a.n + G::TR - 1) / G::TR;
  const int64_t stride = (int64_t)gridDim.x * kVpwLoaders;
  const int64_t tb0 = (int64_t)blockIdx.x * kVpwLoaders;
  const int rounds = tb0 < ntiles ? (int)((ntiles - tb0 + stride - 1) / stride) : 0;
  T* stage = reinterpret_cast<T*>(smem);
  // Both roles run rounds + 1 iterations with one barrier each.  A loader
  // issues the loads of its next tile as soon as the current one is staged,
  // so they are in flight through the barrier and the products; the two
  // loops keep the loaders' registers apart from the accumulators.
  if (loader) {
    V16<T> pg[G::NPASS], px[G::NPASS], pv[G::NPASS];
    auto rows_of = [&](int r) {
      const int64_t t = tb0 + (int64_t)r * stride + wv;
      return t >= ntiles ? 0 : (int)((a.n - t * G::TR) < G::TR ? (a.n - t * G::TR) : G::TR);
    };
    auto fetch = [&](int r) {
      const int64_t r0 = (tb0 + (int64_t)r * stride + wv) * G::TR;
      const int cnt = rows_of(r);
#pragma unroll
      for (int pass = 0; pass < G::NPASS; ++pass) {
        const int gi = pass * G::RPW + g;
        if (gi < cnt) {
          const size_t off = (size_t)(r0 + gi) * KP + j * G::VECN;
          pg[pass] = ld16(static_cast<const T*>(a.G) + off);
          px[pass] = ld16(static_cast<const T*>(a.X) + off);
          if (!first) pv[pass] = ld16(static_cast<const T*>(a.Vp) + off);
        }
      }
    };
    if (rounds > 0) fetch(0);
    for (int r = 0; r <= rounds; ++r) {
      if (r < rounds) {
        const int64_t r0 = (tb0 + (int64_t)r * stride + wv) * G::TR;
        const int cnt = rows_of(r);
        T* tv = stage + (r & 1) * W::BUF + wv * W::AREA;
        T* tx = tv + G::TILE_ELEMS;
#pragma unroll
        for (int pass = 0; pass < G::NPASS; ++pass) {
          const int gi = pass * G::RPW + g;
          const size_t off = (size_t)(r0 + gi) * KP + j * G::VECN;
          V16<T> v, x;
          if (gi < cnt) {
            const V16<T> gv = pg[pass];
            x = px[pass];
            if (!first) {
#pragma unroll
              for (int q = 0; q < G::VECN; ++q) v.v[q] = fma(beta_c[q], pv[pass].v[q], -gv.v[q]);
            } else {
#pragma unroll
              for (int q = 0; q < G::VECN; ++q) v.v[q] = -gv.v[q];
            }
            st16(static_cast<T*>(a.V) + off, v);
            if (a.Vb) st_bf16<KP>(a.Vb, (size_t)(r0 + gi), j, v);
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) cacc[0][q] += (double)v.v[q] * (double)gv.v[q];
          } else {
#pragma unroll
            for (int q = 0; q < G::VECN; ++q) v.v[q] = x.v[q] = T(0);
          }
          tile_store_vec<T, KP>(tv, gi, j, v);
          tile_store_vec<T, KP>(tx, gi, j, x);
        }
        if (r + 1 < rounds) fetch(r + 1);
      }
      __syncthreads();
    }
  } else {
    for (int r = 0; r <= rounds; ++r) {
      if (r > 0) sg.template accumulate<true>(stage + ((r - 1) & 1) * W::BUF, W::AREA, lane);
      __syncthreads();
    }
  }

  double* red = reinterpret_cast<double*>(smem);
  double* prow = a.partials + (size_t)blockIdx.x * a.nv;
  constexpr int KK = KP * KP;
  sg.out(0, true, red, prow, 0, lane);
  sg.out(1, false, red, prow, KK, lane);
  block_vec_out<T, KP, 1>(cacc, red, prow, 2 * KK, wave, lane, kVpwLoaders);
}

// ---------------------------------------------------------------------------
// Deterministic two-level reduction of partial rows:
// out[v] = sum_b partials[b][v], summed in block order.  The first level sums
// groups of kFinChunk rows into lvl2; the second, a launch of its own, sums the
// groups in order.  Two launches instead of one with a last-block ticket: the
// ticket needs a device-scope release in every block, and with one L2 per XCD
// that costs a write-back of dirty L2 lines per block.
// ---------------------------------------------------------------------------

// v < split: out[v]; v >= split: out2[v - split]
__device__ inline void finalize_store(double* out, double* out2, int split, int v, double x) {
  if (v < split) out[v] = x;
  else out2[v - split] = x;
}

__global__ void __launch_bounds__(64) finalize_kernel(const double* __restrict__ partials, int nb,
                                                      int nv, double* __restrict__ lvl2,
                                                      double* __restrict__ out, int split,
                                                      double* __restrict__ out2) {
  const int v = blockIdx.x * 64 + threadIdx.x;
  const int b0 = blockIdx.y * kFinChunk;
  if (v >= nv) return;
  // all loads are issued before any addition; the sum then runs in block order
  double x[kFinChunk];
#pragma unroll
  for (int b = 0; b < kFinChunk; ++b)
    x[b] = (b0 + b < nb) ? partials[(size_t)(b0 + b) * nv + v] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int b = 0; b < kFinChunk; ++b) s += x[b];
  if (gridDim.y == 1) finalize_store(out, out2, split, v, s);
  else lvl2[(size_t)blockIdx.y * nv + v] = s;
}

__global__ void __launch_bounds__(64) finalize2_kernel(const double* __restrict__ lvl2, int ny,
                                                       int nv, double* __restrict__ out, int split,
                                                       double* __restrict__ out2) {
  const int v = blockIdx.x * 64 + threadIdx.x;
  if (v >= nv) return;
  double x[kMaxBlocks / kFinChunk];
#pragma unroll
  for (int y = 0; y < kMaxBlocks / kFinChunk; ++y) x[y] = (y < ny) ? lvl2[(size_t)y * nv + v] : 0.0;
  double t = 0.0;
#pragma unroll
  for (int y = 0; y < kMaxBlocks / kFinChunk; ++y) t += x[y];
  finalize_store(out, out2, split, v, t);
}

// ---------------------------------------------------------------------------
// Exact line search (Section 3.2) in one workgroup, FP64
// ---------------------------------------------------------------------------

struct Roots {
  int n;
  double r[3];
  int mult[3];
};

__device__ inline double cubic_eval(double a3, double a2, double a1, double a0, double x) {
  return ((a3 * x + a2) * x + a1) * x + a0;
}

__device__ inline double newton2(double a3, double a2, double a1, double a0, double x) {
  for (int it = 0; it < 2; ++it) {
    const double dp = (3.0 * a3 * x + 2.0 * a2) * x + a1;
    if (dp == 0.0 || !isfinite(dp)) break;
    const double xn = x - cubic_eval(a3, a2, a1, a0, x) / dp;
    if (!isfinite(xn)) break;
    x = xn;
  }
  return x;
}

__device__ inline void sort_roots(Roots& R) {
  for (int i = 1; i < R.n; ++i)
    for (int k = i; k > 0 && R.r[k] < R.r[k - 1]; --k) {
      const double t = R.r[k];
      R.r[k] = R.r[k - 1];
      R.r[k - 1] = t;
      const int m = R.mult[k];
      R.mult[k] = R.mult[k - 1];
      R.mult[k - 1] = m;
    }
}

// Real roots of a3 x^3 + a2 x^2 + a1 x + a0: Cardano's formula for one real
// root, the trigonometric form for three, the repeated-root closed form when
// the discriminant vanishes (relative tolerance 1e-12); two Newton steps.
__device__ inline Roots cubic_roots(double a3, double a2, double a1, double a0) {
  const double tol = 1e-12;
  Roots R;
  R.n = 0;
  if (a3 == 0.0) {
    if (a2 == 0.0) {
      if (a1 != 0.0) {
        R.n = 1;
        R.r[0] = -a0 / a1;
        R.mult[0] = 1;
      }
      return R;
    }
    const double disc = a1 * a1 - 4.0 * a2 * a0;
    const double scale = fmax(a1 * a1, fabs(4.0 * a2 * a0));
    if (disc < -tol * scale) return R;
    if (disc <= tol * scale) {
      R.n = 1;
      R.r[0] = -a1 / (2.0 * a2);
      R.mult[0] = 2;
      return R;
    }
    const double sq = sqrt(disc);
    const double qq = -0.5 * (a1 + copysign(sq, a1));
    const double r1 = qq / a2;
    const double r2 = (qq != 0.0) ? a0 / qq : -a1 / a2 - r1;
    R.n = 2;
    R.r[0] = r1;
    R.r[1] = r2;
    R.mult[0] = R.mult[1] = 1;
    sort_roots(R);
    return R;
  }
  const double b = a2 / a3, c = a1 / a3, d = a0 / a3;
  const double p = c - b * b / 3.0;
  const double q = 2.0 * b * b * b / 27.0 - b * c / 3.0 + d;
  const double shift = -b / 3.0;
  const double D = q * q / 4.0 + p * p * p / 27.0;
  const double scale = fmax(q * q / 4.0, fabs(p * p * p / 27.0));
  if (scale == 0.0) {
    R.n = 1;
    R.r[0] = newton2(a3, a2, a1, a0, shift);
    R.mult[0] = 3;
    return R;
  }
  if (fabs(D) <= tol * scale) {
    if (p == 0.0) {
      R.n = 1;
      R.r[0] = newton2(a3, a2, a1, a0, shift);
      R.mult[0] = 3;
      return R;
    }
    R.n = 2;
    R.r[0] = newton2(a3, a2, a1, a0, 3.0 * q / p + shift);
    R.mult[0] = 1;
    R.r[1] = -3.0 * q / (2.0 * p) + shift;
    R.mult[1] = 2;
    sort_roots(R);
    return R;
  }
  if (D > 0.0) {
    const double sq = sqrt(D);
    const double u = cbrt(-q / 2.0 + sq);
    const double v = cbrt(-q / 2.0 - sq);
    R.n = 1;
    R.r[0] = newton2(a3, a2, a1, a0, u + v + shift);
    R.mult[0] = 1;
    return R;
  }
  const double m = 2.0 * sqrt(-p / 3.0);
  double arg = 3.0 * q / (p * m);
  arg = fmin(1.0, fmax(-1.0, arg));
  const double th = acos(arg) / 3.0;
  const double two_pi_3 = 2.0943951023931954923;  // 2 pi / 3
  R.n = 3;
  for (int i = 0; i < 3; ++i) {
    R.r[i] = newton2(a3, a2, a1, a0, m * cos(th - two_pi_3 * i) + shift);
    R.mult[i] = 1;
  }
  sort_roots(R);
  return R;
}

// Root rules of Section 3.2: one real root -> it; a simple and a repeated root
// -> the simple one; otherwise the least line objective
// Phi(x) = a3 x^4/4 + a2 x^3/3 + a1 x^2/2 + a0 x (OFM) or the smallest |x|
// (triangular variants).  Candidates are visited by ascending |x| then x, and
// only a strictly smaller Phi replaces the current choice.
__device__ inline double select_root(bool tri, double a3, double a2, double a1, double a0,
                                     int* nroots) {
  Roots R = cubic_roots(a3, a2, a1, a0);
  *nroots = R.n;
  if (R.n == 0) return 0.0;
  if (R.n == 1) return R.r[0];
  if (R.n == 2 && (R.mult[0] == 2 || R.mult[1] == 2)) return R.mult[0] == 1 ? R.r[0] : R.r[1];
  double c[3];
  for (int i = 0; i < R.n; ++i) c[i] = R.r[i];
  for (int i = 1; i < R.n; ++i)
    for (int k = i; k > 0; --k) {
      const bool less = fabs(c[k]) < fabs(c[k - 1]) || (fabs(c[k]) == fabs(c[k - 1]) && c[k] < c[k - 1]);
      if (!less) break;
      const double t = c[k];
      c[k] = c[k - 1];
      c[k - 1] = t;
    }
  if (tri) return c[0];
  double best = c[0];
  double bv = ((a3 * best / 4.0 + a2 / 3.0) * best + a1 / 2.0) * best * best + a0 * best;
  for (int i = 1; i < R.n; ++i) {
    const double x = c[i];
    const double val = ((a3 * x / 4.0 + a2 / 3.0) * x + a1 / 2.0) * x * x + a0 * x;
    if (val < bv) {
      best = x;
      bv = val;
    }
  }
  return best;
}

// deterministic block sum of one double per thread (blockDim = 256)
__device__ inline double block_sum256(double x, double* buf) {
  buf[threadIdx.x] = x;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] += buf[threadIdx.x + s];
    __syncthreads();
  }
  const double r = buf[0];
  __syncthreads();
  return r;
}

// frozen (nullable): once the residual met the tolerance every step size is
// 0, so the iterate that met it is the one kept.  freeze_eps > 0: a step whose
// direction is negligible against the iterate, ||G||_F <= freeze_eps ||X||_F
// (from the column sums diag G^T G of the direction pass and tr X^T X), also
// takes every step size 0.  A cubic that is not identically zero but has no
// real root (Section 3.2 has no rule for it) takes step 0 and sets kStNoRoot.
template <int KP>
__device__ __forceinline__ void linesearch_body(int variant, int first, double alpha0,
                                                double* sc, int* status, const int* frozen,
                                                bool advance_h = false, double freeze_eps = 0.0,
                                                int upper_fd = 0) {
  bool frz = frozen != nullptr && *frozen != 0;
  __shared__ double buf[256];
  __shared__ double co[4];
  const int KK = KP * KP;
  const double* M = sc + SC<KP>::M;
  if (upper_fd == 1) {
    // diag(V^T A V)_c = -(V^T V)_cc - 2 sum_i V_ic sum_{j in copy row i} w_ij V_jc
    const int t = threadIdx.x;
    if (t < KP) sc[SC<KP>::FD + t] = -sc[SC<KP>::P + t * KP + t] - 2.0 * sc[SC<KP>::FD + t];
    __syncthreads();
  } else if (upper_fd == 2) {
    // V^T A V = -V^T V - (S + S^T), S = sum_i V_i^T sum_{j in copy row i} w_ij V_j;
    // each pair (r, c), (c, r) is rewritten by one thread
    double* F = sc + SC<KP>::F;
    const double* P = sc + SC<KP>::P;
    for (int e = threadIdx.x; e < KK; e += blockDim.x) {
      const int r = e / KP, c = e % KP;
      if (r <= c) {
        const double w = F[r * KP + c] + F[c * KP + r];
        F[r * KP + c] = -P[r * KP + c] - w;
        F[c * KP + r] = -P[c * KP + r] - w;
      }
    }
    __syncthreads();
  }
  if (freeze_eps > 0.0) {
    const int t = threadIdx.x;
    const double g2 = block_sum256(t < KP ? sc[SC<KP>::GG + t] : 0.0, buf);
    const double x2 = block_sum256(t < KP ? M[t * KP + t] : 0.0, buf);
    if (sqrt(g2) <= freeze_eps * sqrt(x2)) frz = true;
  }
  const double* H = sc + SC<KP>::H;
  const double* C = sc + SC<KP>::C;
  const double* P = sc + SC<KP>::P;
  const double* E = sc + SC<KP>::E;
  const double* F = sc + SC<KP>::F;
  const double* vg = sc + SC<KP>::VG;
  const double* fd = sc + SC<KP>::FD;
  double* alpha = sc + SC<KP>::ALPHA;
  double* coef = sc + SC<KP>::COEF;
  double* nroot = sc + SC<KP>::NROOT;
  const int tid = threadIdx.x;
  const bool tri = (variant == OFM_TRI_F1 || variant == OFM_TRI_F2);
  bool bad = false;

  if (!tri) {
    // traces tr(X Y) = sum_ab X_ab Y_ba
    double t3 = 0.0, t2 = 0.0, t1 = 0.0;
    for (int e = tid; e < KK; e += 256) {
      const int r = e / KP, c = e % KP;
      const int et = c * KP + r;
      if (variant == OFM_F1) {
        t3 += P[e] * P[et];                                     // tr(P P)
        t2 += P[e] * C[et];                                     // tr(P C)
        t1 += C[et] * C[e] + C[et] * C[et] + P[e] * M[et];      // tr(C^T C^T) + tr(C^T C) + tr(P M)
      } else {
        t3 += P[e] * F[et];                                     // tr(P F)
        t2 += C[et] * F[et] + P[e] * E[e];                      // tr(C^T F) + tr(P E^T)
        t1 += 2.0 * C[et] * E[et] + 2.0 * C[et] * E[e] + P[e] * H[et] + M[e] * F[et];
      }
    }
    double tr_f = 0.0, svg = 0.0;
    if (tid < KP) {
      tr_f = (variant == OFM_F1) ? fd[tid] : F[tid * KP + tid];
      svg = vg[tid];
    }
    t3 = block_sum256(t3, buf);
    t2 = block_sum256(t2, buf);
    t1 = block_sum256(t1, buf);
    tr_f = block_sum256(tr_f, buf);
    svg = block_sum256(svg, buf);
    if (tid == 0) {
      double a3, a2, a1, a0;
      if (variant == OFM_F1) {
        // (1/4) d/da f1(X + aV), eq. f1-derivative
        a3 = t3;
        a2 = 3.0 * t2;
        a1 = tr_f + t1;
        a0 = svg / 4.0;
      } else {
        // d/da f2(X + aV), eq. f2-derivative
        a3 = -4.0 * t3;
        a2 = -6.0 * t2;
        a1 = 2.0 * (2.0 * tr_f - t1);
        a0 = svg;
      }
      co[0] = a3;
      co[1] = a2;
      co[2] = a1;
      co[3] = a0;
      int nr = 0;
      double al = first ? alpha0 : select_root(false, a3, a2, a1, a0, &nr);
      if (!(isfinite(a3) && isfinite(a2) && isfinite(a1) && isfinite(a0) && isfinite(al))) {
        bad = true;
        al = 0.0;
      }
      if (!first && nr == 0 && (a3 != 0.0 || a2 != 0.0 || a1 != 0.0 || a0 != 0.0))
        atomicOr(status, kStNoRoot);
      if (frz) al = 0.0;
      coef[0] = a3;
      coef[1] = a2;
      coef[2] = a1;
      coef[3] = a0;
      nroot[0] = nr;
      buf[0] = al;
      if (bad) atomicOr(status, kStNonfinite);
    }
    __syncthreads();
    const double al = buf[0];
    if (tid < KP) alpha[tid] = al;
    if (tid > 0 && tid < KP) {
      for (int jj = 0; jj < 4; ++jj) coef[4 * tid + jj] = 0.0;
      nroot[tid] = 0;
    }
  } else if (tid < KP) {
    // per-column cubic [V^T g(X + a_i V)]_ii, eqs. alphai-f1 / alphai-f2:
    // [X triu(Y)]_ii = sum_{j<=i} X_ij Y_ji
    const int i = tid;
    double a3 = 0.0, a2 = 0.0, a1 = 0.0;
    for (int jj = 0; jj <= i; ++jj) {
      const int ij = i * KP + jj, ji = jj * KP + i;
      if (variant == OFM_TRI_F1) {
        a3 += P[ij] * P[ji];
        a2 += P[ij] * C[ji] + P[ij] * C[ij] + C[ji] * P[ji];
        a1 += C[ji] * C[ij] + C[ji] * C[ji] + P[ij] * M[ji];
      } else {
        a3 -= F[ij] * P[ji] + P[ij] * F[ji];
        a2 -= E[ji] * P[ji] + F[ij] * C[ji] + F[ij] * C[ij] + C[ji] * F[ji] + P[ij] * E[ji] +
              P[ij] * E[ij];
        a1 -= E[ji] * C[ji] + E[ji] * C[ij] + F[ij] * M[ji] + C[ji] * E[ji] + C[ji] * E[ij] +
              P[ij] * H[ji];
      }
    }
    if (variant == OFM_TRI_F1) a1 += fd[i];
    else a1 += 2.0 * F[i * KP + i];
    const double a0 = vg[i];
    int nr = 0;
    double al = first ? alpha0 : select_root(true, a3, a2, a1, a0, &nr);
    if (!(isfinite(a3) && isfinite(a2) && isfinite(a1) && isfinite(a0) && isfinite(al))) {
      atomicOr(status, kStNonfinite);
      al = 0.0;
    }
    if (!first && nr == 0 && (a3 != 0.0 || a2 != 0.0 || a1 != 0.0 || a0 != 0.0))
      atomicOr(status, kStNoRoot);
    if (frz) al = 0.0;
    coef[4 * i + 0] = a3;
    coef[4 * i + 1] = a2;
    coef[4 * i + 2] = a1;
    coef[4 * i + 3] = a0;
    nroot[i] = nr;
    alpha[i] = al;
  }
  // the CG denominator of the next step: diag G^T G of this step
  __syncthreads();
  if (tid < KP) sc[SC<KP>::GGP + tid] = sc[SC<KP>::GG + tid];
  if (advance_h) {
    // H of the next iterate, (X + V D)^T A (X + V D) with D = diag(alpha):
    // H_ij + alpha_j E_ij + alpha_i E_ji + alpha_i alpha_j F_ij (A symmetric,
    // so V^T A X = E^T); each entry is read and written by one thread
    double* Hn = sc + SC<KP>::H;
    for (int e = tid; e < KK; e += 256) {
      const int r = e / KP, c = e % KP;
      const double ar = alpha[r], ac = alpha[c];
      Hn[e] += ac * E[e] + ar * E[c * KP + r] + ar * ac * F[e];
    }
  }
}

template <int KP>
__global__ void __launch_bounds__(256) linesearch_kernel(int variant, int first, double alpha0,
                                                         int advance_h, int upper_fd, double* sc,
                                                         int* status, const int* frozen,
                                                         double freeze_eps) {
  linesearch_body<KP>(variant, first, alpha0, sc, status, frozen, advance_h != 0, freeze_eps,
                      upper_fd);
}

// The root rules of the line search on caller-given cubics (diagnostics):
// coef[4 i + j] = a_{3-j} of cubic i, the same device code as the step.
__global__ void __launch_bounds__(256) select_roots_kernel(int tri, int64_t count,
                                                           const double* __restrict__ coef,
                                                           double* __restrict__ alpha,
                                                           int32_t* __restrict__ nroots) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int nr = 0;
  const double* c = coef + 4 * i;
  alpha[i] = select_root(tri != 0, c[0], c[1], c[2], c[3], &nr);
  nroots[i] = nr;
}

// ---------------------------------------------------------------------------
// Residual of the Ritz pairs of A on span(X) from M = X^T X, H = X^T A X,
// K = (AX)^T (AX):  relres^2 = tr(M^{-1} K) / tr((M^{-1} H)^2) - 1
// (numerical results section, "Evaluation metrics"); also the objective.
// ---------------------------------------------------------------------------

// tol > 0 and frozen != nullptr: a residual <= tol sets *frozen
template <int KP>
__device__ __forceinline__ void residual_body(int variant, double normA2, double* sc,
                                              int* status, double tol, int* frozen) {
  // L: Cholesky factor of M; W: [K | H] side by side (KP x 2KP)
  __shared__ double L[KP * KP];
  __shared__ double W[KP * 2 * KP];
  __shared__ double buf[256];
  __shared__ int fail;
  const int tid = threadIdx.x;
  const int KK = KP * KP;
  constexpr int W2 = 2 * KP;
  const double* M = sc + SC<KP>::M;
  const double* H = sc + SC<KP>::H;
  const double* K = sc + SC<KP>::K;
  for (int e = tid; e < KK; e += 256) {
    L[e] = M[e];
    const int r = e / KP, c = e % KP;
    W[r * W2 + c] = K[e];
    W[r * W2 + KP + c] = H[e];
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  // an exactly zero column of X (a zero-padded width) has a zero row and
  // column in M, H and K; a unit pivot there leaves it out of both traces
  if (tid < KP && L[tid * KP + tid] == 0.0) L[tid * KP + tid] = 1.0;
  __syncthreads();
  // Cholesky M = L L^T by outer products on the unscaled columns: step c
  // subtracts A_rc A_qc / A_cc from the trailing lower triangle (one barrier
  // per step), leaving A_rc (r >= c) as it stood at step c.  The factor is
  // then L_cc = sqrt(A_cc), L_rc = A_rc / sqrt(A_cc), so L_rc / L_cc =
  // A_rc / A_cc: kept in place of L below the diagonal, with 1 / L_rr in rd.
  __shared__ double rd[KP];
  for (int c = 0; c < KP; ++c) {
    const double d = L[c * KP + c];
    const double inv = 1.0 / ((d > 0.0) ? d : 1.0);
    if (tid == 0 && (!(d > 0.0) || !isfinite(d))) fail = 1;
    const int m = KP - 1 - c;
    for (int e = tid; e < m * m; e += 256) {
      const int r = c + 1 + e / m, q = c + 1 + e % m;
      if (q <= r) L[r * KP + q] -= L[r * KP + c] * L[q * KP + c] * inv;
    }
    __syncthreads();
  }
  if (tid < KP) {
    const double d = L[tid * KP + tid];
    buf[tid] = 1.0 / ((d > 0.0) ? d : 1.0);
    rd[tid] = 1.0 / ((d > 0.0) ? sqrt(d) : 1.0);
  }
  __syncthreads();
  for (int e = tid; e < KK; e += 256) {
    const int r = e / KP, c = e % KP;
    if (r > c) L[e] *= buf[c];
  }
  __syncthreads();
  // With M = L L^T: tr(M^{-1} K) = tr(L^{-1} K L^{-T}) and tr((M^{-1} H)^2) =
  // ||L^{-1} H L^{-T}||_F^2 (K, H symmetric).  Both by two forward
  // substitutions with a transpose between them.  A substitution eliminates
  // one row at a time on unscaled rows, z_r -= (L_rq / L_qq) z_q (one barrier
  // per row, every thread updating the rows below), and scales row r by
  // 1 / L_rr at the end.
  for (int half = 0; half < 2; ++half) {
    for (int q = 0; q < KP - 1; ++q) {
      for (int e = tid; e < (KP - 1 - q) * W2; e += 256) {
        const int r = q + 1 + e / W2, c = e % W2;
        W[r * W2 + c] -= L[r * KP + q] * W[q * W2 + c];
      }
      __syncthreads();
    }
    for (int e = tid; e < KP * W2; e += 256) W[e] *= rd[e / W2];
    __syncthreads();
    if (half == 0) {
      // in-place transpose of each block: (L^{-1} B)^T = B L^{-T}
      for (int e = tid; e < 2 * KK; e += 256) {
        const int b = e / KK, r = (e % KK) / KP, c = e % KP;
        if (c > r) {
          const double x = W[r * W2 + b * KP + c];
          W[r * W2 + b * KP + c] = W[c * W2 + b * KP + r];
          W[c * W2 + b * KP + r] = x;
        }
      }
      __syncthreads();
    }
  }
  double pk = 0.0, ph = 0.0;
  if (tid < KP) pk = W[tid * W2 + tid];
  for (int e = tid; e < KK; e += 256) {
    const double x = W[(e / KP) * W2 + KP + e % KP];
    ph += x * x;
  }
  const double trMK = block_sum256(pk, buf);
  const double trMH2 = block_sum256(ph, buf);
  // objective: f1 = ||A||^2 + 2 tr(H) + ||M||_F^2 ; f2 = 2 tr(H) - tr(M H)
  double trH = (tid < KP) ? H[tid * KP + tid] : 0.0;
  double mm = 0.0;
  for (int e = tid; e < KK; e += 256) {
    const int r = e / KP, q = e % KP;
    mm += (variant == OFM_F1 || variant == OFM_TRI_F1) ? M[e] * M[e] : M[e] * H[q * KP + r];
  }
  trH = block_sum256(trH, buf);
  mm = block_sum256(mm, buf);
  if (tid == 0) {
    const double rr = trMK / trMH2 - 1.0;
    sc[SC<KP>::RELRES] = sqrt(fmax(rr, 0.0));
    sc[SC<KP>::FVAL] = (variant == OFM_F1 || variant == OFM_TRI_F1) ? normA2 + 2.0 * trH + mm
                                                                     : 2.0 * trH - mm;
    if (fail) atomicOr(status, kStCholesky);
    if (!isfinite(sc[SC<KP>::RELRES])) atomicOr(status, kStNonfinite);
    if (frozen != nullptr && tol > 0.0 && !fail && sc[SC<KP>::RELRES] <= tol) *frozen = 1;
  }
}

template <int KP>
__global__ void __launch_bounds__(256) residual_kernel(int variant, double normA2, double* sc,
                                                       int* status, double tol, int* frozen) {
  residual_body<KP>(variant, normA2, sc, status, tol, frozen);
}

// objective from the k x k products only: f1 = ||A||_F^2 + 2 tr(H) + ||M||_F^2,
// f2 = 2 tr(H) - tr(M H)
template <int KP>
__global__ void __launch_bounds__(256) objective_kernel(int variant, double normA2,
                                                       const double* __restrict__ sc,
                                                       double* __restrict__ out) {
  __shared__ double buf[256];
  const int tid = threadIdx.x;
  const double* M = sc + SC<KP>::M;
  const double* H = sc + SC<KP>::H;
  const bool f1 = (variant == OFM_F1 || variant == OFM_TRI_F1);
  double trH = (tid < KP) ? H[tid * KP + tid] : 0.0;
  double mm = 0.0;
  for (int e = tid; e < KP * KP; e += 256) {
    const int r = e / KP, q = e % KP;
    mm += f1 ? M[e] * M[e] : M[e] * H[q * KP + r];
  }
  trH = block_sum256(trH, buf);
  mm = block_sum256(mm, buf);
  if (tid == 0) out[0] = f1 ? normA2 + 2.0 * trH + mm : 2.0 * trH - mm;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

template <typename T, int KP>
int tile_rows_t() {
  return Geo<T, KP>::TR;
}

int tile_rows(int precision, int k) {
  const bool d = precision == OFM_FP64;
  switch (k) {
    case 4: return d ? tile_rows_t<double, 4>() : tile_rows_t<float, 4>();
    case 8: return d ? tile_rows_t<double, 8>() : tile_rows_t<float, 8>();
    case 16: return d ? tile_rows_t<double, 16>() : tile_rows_t<float, 16>();
    case 32: return d ? tile_rows_t<double, 32>() : tile_rows_t<float, 32>();
    case 64: return d ? 16 : tile_rows_t<float, 64>();
  }
  return 16;
}

template <typename T, int KP>
int wpb_t() {
  return Cfg<T, KP>::WPB;
}

static int wpb(int precision, int k) {
  const bool d = precision == OFM_FP64;
  switch (k) {
    case 4: return d ? wpb_t<double, 4>() : wpb_t<float, 4>();
    case 8: return d ? wpb_t<double, 8>() : wpb_t<float, 8>();
    case 16: return d ? wpb_t<double, 16>() : wpb_t<float, 16>();
    case 32: return d ? wpb_t<double, 32>() : wpb_t<float, 32>();
    case 64: return wpb_t<float, 64>();
  }
  return 1;
}

int spmm_wpb(int precision, int k) { return wpb(precision, k); }

int pass_blocks(int precision, int k, int64_t ntiles) {
  const int w = wpb(precision, k);
  int64_t nb = (ntiles + w - 1) / w;
  if (nb > kMaxBlocks) nb = kMaxBlocks;
  if (nb < 1) nb = 1;
  return (int)nb;
}

int partial_nv(int k, int mode, int flags) {
  switch (k) {
    case 4: return mode_nv<4>(mode, flags);
    case 8: return mode_nv<8>(mode, flags);
    case 16: return mode_nv<16>(mode, flags);
    case 32: return mode_nv<32>(mode, flags);
    case 64: return mode_nv<64>(mode, flags);
  }
  return 0;
}

int partial_off(int k, int mode) {
  switch (k) {
    case 4: return mode_off<4>(mode);
    case 8: return mode_off<8>(mode);
    case 16: return mode_off<16>(mode);
    case 32: return mode_off<32>(mode);
    case 64: return mode_off<64>(mode);
  }
  return 0;
}

// Workgroups of a kernel the chip holds at once (occupancy x CUs), taken at
// its first launch.  The passes are grid-stride loops with equal work per
// workgroup, so a grid that is not a whole number of such rounds ends with a
// short round at low occupancy; launch_rounded trims the grid to whole rounds.
template <auto Kernel>
static int resident_blocks(int threads, int smem) {
  static const int cap = [&] {
    int occ = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, Kernel, threads, smem) != hipSuccess ||
        hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    return occ * cus;
  }();
  return cap;
}

template <auto Kernel>
static hipError_t launch_rounded(PassArgs& a, int threads, int smem, hipStream_t s) {
  const int cap = resident_blocks<Kernel>(threads, smem);
  // the XCD slots rely on the grid as given (in-order dispatch, a multiple of 8)
  if (!a.xcd && cap > 0 && a.nblocks > cap) a.nblocks = (a.nblocks / cap) * cap;
  hipLaunchKernelGGL(Kernel, dim3(a.nblocks), dim3(threads), smem, s, a);
  return hipGetLastError();
}

template <typename T, int KP, int MODE, bool BF, bool HC>
static hipError_t spmm_mode_bf(PassArgs& a, hipStream_t s) {
  using SM = Smem<T, KP, MODE>;
  // the k x k products of the residual (X^T A X, (AX)^T (AX)) are compiled in
  // only for the iterations that check it; those keep the default gather
  // policy (at their lower occupancy the hot/cold form measured slower)
  if ((MODE == kGF1 || MODE == kGF2 || MODE == kAXF2) && (a.flags & kFlagCheck))
    return launch_rounded<spmm_kernel<T, KP, MODE, true, BF, false>>(a, SM::WPB * 64, SM::bytes,
                                                                      s);
  return launch_rounded<spmm_kernel<T, KP, MODE, false, BF, HC>>(a, SM::WPB * 64, SM::bytes, s);
}

template <typename T, int KP, int MODE>
static hipError_t spmm_mode(PassArgs& a, hipStream_t s) {
  if constexpr (sizeof(T) == 4 && MODE != kApply) {
    if (a.Zg) return spmm_mode_bf<T, KP, MODE, true, false>(a, s);
  }
  if (a.flags & kFlagHC) return spmm_mode_bf<T, KP, MODE, false, true>(a, s);
  return spmm_mode_bf<T, KP, MODE, false, false>(a, s);
}

template <typename T, int KP>
static hipError_t spmm_t(PassArgs& a, hipStream_t s) {
  switch (a.mode) {
    case kApply: return spmm_mode<T, KP, kApply>(a, s);
    case kGF1: return spmm_mode<T, KP, kGF1>(a, s);
    case kGF2: return spmm_mode<T, KP, kGF2>(a, s);
    case kAXF2: return spmm_mode<T, KP, kAXF2>(a, s);
    case kAVF1: return spmm_mode<T, KP, kAVF1>(a, s);
    case kAVF2: return spmm_mode<T, KP, kAVF2>(a, s);
    case kSF2:
      if constexpr (KP <= 32) return spmm_mode<T, KP, kSF2>(a, s);
      break;
  }
  return hipErrorInvalidValue;
}

template <typename T, int KP, int MODE>
static hipError_t dense_mode(PassArgs& a, hipStream_t s) {
  using SM = Smem<T, KP, MODE>;
  if constexpr (sizeof(T) == 4 && KP == 64 && MODE == kVPass)
    return launch_rounded<vpass_ws_kernel>(a, 2 * kVpwLoaders * 64, VPassWS::bytes, s);
  else
    return launch_rounded<dense_kernel<T, KP, MODE>>(a, SM::WPB * 64, SM::bytes, s);
}

template <typename T, int KP>
static hipError_t dense_t(PassArgs& a, hipStream_t s) {
  switch (a.mode) {
    case kGPassF2: return dense_mode<T, KP, kGPassF2>(a, s);
    case kGPassF1: return dense_mode<T, KP, kGPassF1>(a, s);
    case kVPass: return dense_mode<T, KP, kVPass>(a, s);
    case kVPassE:
      if constexpr (KP <= 32) return dense_mode<T, KP, kVPassE>(a, s);
      break;
    case kUpdate: return dense_mode<T, KP, kUpdate>(a, s);
    case kUpdateR: return dense_mode<T, KP, kUpdateR>(a, s);
    case kGramM: return dense_mode<T, KP, kGramM>(a, s);
    case kGGP: return dense_mode<T, KP, kGGP>(a, s);
    case kEF: return dense_mode<T, KP, kEF>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_spmm(int precision, int k, PassArgs& a, hipStream_t s) {
  if (precision == OFM_FP64) {
    switch (k) {
      case 4: return spmm_t<double, 4>(a, s);
      case 8: return spmm_t<double, 8>(a, s);
      case 16: return spmm_t<double, 16>(a, s);
      case 32: return spmm_t<double, 32>(a, s);
    }
  } else {
    switch (k) {
      case 4: return spmm_t<float, 4>(a, s);
      case 8: return spmm_t<float, 8>(a, s);
      case 16: return spmm_t<float, 16>(a, s);
      case 32: return spmm_t<float, 32>(a, s);
      case 64: return spmm_t<float, 64>(a, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_dense(int precision, int k, PassArgs& a, hipStream_t s) {
  if (precision == OFM_FP64) {
    switch (k) {
      case 4: return dense_t<double, 4>(a, s);
      case 8: return dense_t<double, 8>(a, s);
      case 16: return dense_t<double, 16>(a, s);
      case 32: return dense_t<double, 32>(a, s);
    }
  } else {
    switch (k) {
      case 4: return dense_t<float, 4>(a, s);
      case 8: return dense_t<float, 8>(a, s);
      case 16: return dense_t<float, 16>(a, s);
      case 32: return dense_t<float, 32>(a, s);
      case 64: return dense_t<float, 64>(a, s);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const double* partials, int nb, int nv, double* out, double* lvl2,
                           hipStream_t s, int split, double* out2) {
  if (split >= nv || !out2) {
    split = nv;
    out2 = out;
  }
  const int nx = (nv + 63) / 64;
  // more partial rows than one two-level pass takes: sum groups of kFinChunk
  // rows level by level (in block order) into lvl2 and the region after it
  // (lvl2 holds ceil(nb / kFinChunk) + ceil(nb / kFinChunk^2) rows of nv)
  if (nb > kMaxBlocks) {
    double* buf[2] = {lvl2, lvl2 + (size_t)((nb + kFinChunk - 1) / kFinChunk) * nv};
    int w = 0;
    while (nb > kMaxBlocks) {
      const int ny = (nb + kFinChunk - 1) / kFinChunk;
      hipLaunchKernelGGL(finalize_kernel, dim3(nx, ny), dim3(64), 0, s, partials, nb, nv, buf[w],
                         out, split, out2);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      partials = buf[w];
      nb = ny;
      w ^= 1;
    }
    lvl2 = buf[w];
  }
  const int ny = (nb + kFinChunk - 1) / kFinChunk;
  hipLaunchKernelGGL(finalize_kernel, dim3(nx, ny), dim3(64), 0, s, partials, nb, nv, lvl2, out,
                     split, out2);
  if (ny > 1) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize2_kernel, dim3(nx), dim3(64), 0, s, lvl2, ny, nv, out, split, out2);
  }
  return hipGetLastError();
}

hipError_t launch_linesearch(int k, int variant, int first, double alpha0, int advance_h,
                             int upper_fd, double* sc, int* status, const int* frozen,
                             double freeze_eps, hipStream_t s) {
#define OFM_LS(KP)                                                                              \
  hipLaunchKernelGGL(linesearch_kernel<KP>, dim3(1), dim3(256), 0, s, variant, first, alpha0, \
                     advance_h, upper_fd, sc, status, frozen, freeze_eps);                     \
  break;
  switch (k) {
    case 4: OFM_LS(4)
    case 8: OFM_LS(8)
    case 16: OFM_LS(16)
    case 32: OFM_LS(32)
    case 64: OFM_LS(64)
    default: return hipErrorInvalidValue;
  }
#undef OFM_LS
  return hipGetLastError();
}

hipError_t launch_select_roots(int tri, int64_t count, const double* coef, double* alpha,
                               int32_t* nroots, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(select_roots_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     tri, count, coef, alpha, nroots);
  return hipGetLastError();
}

hipError_t launch_objective(int k, int variant, double normA2, const double* sc, double* out,
                            hipStream_t s) {
  switch (k) {
    case 4: hipLaunchKernelGGL(objective_kernel<4>, dim3(1), dim3(256), 0, s, variant, normA2, sc, out); break;
    case 8: hipLaunchKernelGGL(objective_kernel<8>, dim3(1), dim3(256), 0, s, variant, normA2, sc, out); break;
    case 16: hipLaunchKernelGGL(objective_kernel<16>, dim3(1), dim3(256), 0, s, variant, normA2, sc, out); break;
    case 32: hipLaunchKernelGGL(objective_kernel<32>, dim3(1), dim3(256), 0, s, variant, normA2, sc, out); break;
    case 64: hipLaunchKernelGGL(objective_kernel<64>, dim3(1), dim3(256), 0, s, variant, normA2, sc, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_residual(int k, int variant, double normA2, double* sc, int* status,
                           double tol, int* frozen, hipStream_t s) {
  switch (k) {
    case 4: hipLaunchKernelGGL(residual_kernel<4>, dim3(1), dim3(256), 0, s, variant, normA2, sc, status, tol, frozen); break;
    case 8: hipLaunchKernelGGL(residual_kernel<8>, dim3(1), dim3(256), 0, s, variant, normA2, sc, status, tol, frozen); break;
    case 16: hipLaunchKernelGGL(residual_kernel<16>, dim3(1), dim3(256), 0, s, variant, normA2, sc, status, tol, frozen); break;
    case 32: hipLaunchKernelGGL(residual_kernel<32>, dim3(1), dim3(256), 0, s, variant, normA2, sc, status, tol, frozen); break;
    case 64: hipLaunchKernelGGL(residual_kernel<64>, dim3(1), dim3(256), 0, s, variant, normA2, sc, status, tol, frozen); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched passes.  Block b is worker b / 8 of XCD b % 8 (workgroups are
// dispatched to the XCDs round-robin); the workers of an XCD sweep the graphs
// assigned to it one after another, each graph's tiles split over all the
// XCD's workers, so an XCD touches one or two graphs' rows at a time and a
// small graph's rows stay in that XCD's L2.  Converged graphs are skipped.
// ---------------------------------------------------------------------------

__device__ inline PassArgs batch_pass_args(const BatchArgs& b, const BatchGraph& d) {
  PassArgs a;
  a.n = d.n;
  a.k = b.k;
  a.mode = b.mode;
  a.variant = b.variant;
  a.flags = b.flags;
  a.sc = d.sc;
  a.partials = d.partials;
  a.nv = b.nv;
  a.status = d.status;
  a.sched = d.sched;
  a.sptr = d.sptr;
  a.tiles = d.tiles;
  a.ntiles = d.ntiles;
  a.pk = d.pk;
  const int cur = b.cur, prev = b.cur ^ 1;
  const bool first = (b.flags & kFlagFirst) != 0;
  switch (b.mode) {
    case kGF1:
      a.Z = d.X;
      a.Zg = b.bf16 ? d.Xb : nullptr;
      a.G = d.G[cur];
      a.Gp = first ? nullptr : d.G[prev];
      a.Vp = first ? nullptr : d.V[prev];
      break;
    case kAXF2:
      a.Z = d.X;
      a.Zg = b.bf16 ? d.Xb : nullptr;
      a.Y = d.AX;
      break;
    case kGPassF2:
    case kGPassF1:
      a.X = d.X;
      a.AX = d.AX;
      a.G = d.G[cur];
      a.Gp = first ? nullptr : d.G[prev];
      a.Vp = first ? nullptr : d.V[prev];
      break;
    case kVPass:
      a.G = d.G[cur];
      a.Vp = first ? nullptr : d.V[prev];
      a.V = d.V[cur];
      a.Vb = b.bf16 ? d.Vb : nullptr;
      a.X = d.X;
      break;
    case kAVF1:
    case kAVF2:
      a.Z = d.V[cur];
      a.Zg = b.bf16 ? d.Vb : nullptr;
      a.X = d.X;
      a.Y = d.AV;
      if (b.mode == kAVF1 && (b.flags & kFlagUpper)) {
        if (d.upk) {
          // the upper-triangle copy, over the workers the full graph uses
          a.sched = d.usched;
          a.sptr = d.usptr;
          a.tiles = d.utiles;
          a.ntiles = d.untiles;
          a.pk = d.upk;
          a.Y = nullptr;
        } else {
          a.flags &= ~kFlagUpper;
        }
      }
      break;
    case kUpdate:
      a.X = d.X;
      a.Xw = d.X;
      a.Xb = b.bf16 ? d.Xb : nullptr;
      a.V = d.V[cur];
      break;
    case kUpdateR:
      a.X = d.X;
      a.Xw = d.X;
      a.Xb = b.bf16 ? d.Xb : nullptr;
      a.V = d.V[cur];
      a.Z = d.AV;
      a.AX = d.AX;
      a.Y = d.AX;
      break;
    case kGramM:
      a.X = d.X;
      a.Xb = b.bf16 ? d.Xb : nullptr;
      break;
  }
  return a;
}

// The graphs of one XCD take consecutive ranges of its workers, wrapping
// around: graph i uses the nw_i workers that start where graph i-1's ended, so
// small graphs run side by side instead of all on the first workers.  Returns
// worker w's rank within the range that starts at base (>= nw: not in it).
__device__ __host__ inline int batch_worker_rank(int w, int base, int workers) {
  const int r = w - base;
  return r >= 0 ? r : r + workers;
}

// workers a graph uses: enough for about tpw tiles per wavefront
__device__ __host__ inline int batch_graph_workers(int64_t ntiles, int wpb, int tpw, int workers) {
  const int64_t per = (int64_t)wpb * tpw;
  const int64_t w = (ntiles + per - 1) / per;
  return (int)(w < 1 ? 1 : (w > workers ? workers : w));
}

// the share of workgroup blk of a batched SpMM pass (blk = blockIdx.x of the
// per-pass launch, or of the persistent launch)
template <int KP, int MODE, bool CHECK, bool BF>
__device__ __forceinline__ void batch_spmm_run(const BatchArgs& b, int blk, unsigned char* smem) {
  const int x = blk & 7;
  const int w = blk >> 3;
  int base = 0;
  for (int i = b.xoff[x]; i < b.xoff[x + 1]; ++i) {
    const BatchGraph& d = b.graphs[b.xlist[i]];
    const int nw = batch_graph_workers(d.ntiles, Cfg<float, KP>::WPB, b.tpw, b.workers);
    const int rank = batch_worker_rank(w, base, b.workers);
    base = (base + nw) % b.workers;
    if (rank >= nw || *d.active == 0) continue;
    const PassArgs a = batch_pass_args(b, d);
    spmm_body<float, KP, MODE, CHECK, BF>(a, rank, nw, smem);
    __syncthreads();
  }
}

template <int KP, int MODE, bool CHECK, bool BF>
__global__ void __launch_bounds__((Cfg<float, KP>::WPB * 64)) batch_spmm_kernel(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  batch_spmm_run<KP, MODE, CHECK, BF>(b, blockIdx.x, smem);
}

template <int KP, int MODE>
__device__ __forceinline__ void batch_dense_run(const BatchArgs& b, int blk, unsigned char* smem) {
  const int x = blk & 7;
  const int w = blk >> 3;
  int base = 0;
  for (int i = b.xoff[x]; i < b.xoff[x + 1]; ++i) {
    const BatchGraph& d = b.graphs[b.xlist[i]];
    const int nw = batch_graph_workers(d.ntiles, Cfg<float, KP>::WPB, b.tpw, b.workers);
    const int rank = batch_worker_rank(w, base, b.workers);
    base = (base + nw) % b.workers;
    if (rank >= nw || *d.active == 0) continue;
    const PassArgs a = batch_pass_args(b, d);
    dense_body<float, KP, MODE>(a, rank, nw, smem);
    __syncthreads();
  }
}

template <int KP, int MODE>
__global__ void __launch_bounds__((Cfg<float, KP>::WPB * 64)) batch_dense_kernel(BatchArgs b) {
  extern __shared__ __align__(16) unsigned char smem[];
  batch_dense_run<KP, MODE>(b, blockIdx.x, smem);
}

// Per-graph sum of its block partial rows, in block order: rows are summed in
// groups of kFinChunk (blockIdx.z = group); with more than one group the group
// sums go to the graph's lvl2 rows and batch_finalize2_kernel adds them in
// order, which keeps several waves per graph in flight.
template <int KP>
__device__ inline void batch_store(const BatchArgs& b, const BatchGraph& d, int v, double s) {
  // the update of the recurrence writes [M | H]: H goes to its own slot
  const int split = (b.mode == kUpdateR && (b.flags & kFlagH)) ? KP * KP : b.nv;
  d.sc[v < split ? b.off + v : SC<KP>::H + (v - split)] = s;
}

// (bx, by, bz): the 64-lane block of the per-pass launch's grid, lane < 64
template <int KP>
__device__ inline void batch_finalize_run(const BatchArgs& b, int bx, int by, int bz, int lane) {
  const BatchGraph& d = b.graphs[by];
  if (*d.active == 0) return;
  const int v = bx * 64 + lane;
  if (v >= b.nv) return;
  const int nw = batch_graph_workers(d.ntiles, Cfg<float, KP>::WPB, b.tpw, b.workers);
  const int ng = (nw + kFinChunk - 1) / kFinChunk;
  const int b0 = bz * kFinChunk;
  if (b0 >= nw) return;
  double x[kFinChunk];
#pragma unroll
  for (int q = 0; q < kFinChunk; ++q)
    x[q] = (b0 + q < nw) ? d.partials[(size_t)(b0 + q) * b.nv + v] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kFinChunk; ++q) s += x[q];
  if (ng == 1) batch_store<KP>(b, d, v, s);
  else d.lvl2[(size_t)bz * b.nv + v] = s;
}

template <int KP>
__global__ void __launch_bounds__(64) batch_finalize_kernel(BatchArgs b) {
  batch_finalize_run<KP>(b, blockIdx.x, blockIdx.y, blockIdx.z, threadIdx.x);
}

template <int KP>
__device__ inline void batch_finalize2_run(const BatchArgs& b, int bx, int by, int lane) {
  const BatchGraph& d = b.graphs[by];
  if (*d.active == 0) return;
  const int v = bx * 64 + lane;
  if (v >= b.nv) return;
  const int nw = batch_graph_workers(d.ntiles, Cfg<float, KP>::WPB, b.tpw, b.workers);
  const int ng = (nw + kFinChunk - 1) / kFinChunk;
  if (ng == 1) return;
  constexpr int G = (kBatchMaxWorkers + kFinChunk - 1) / kFinChunk;
  double x[G];
#pragma unroll
  for (int y = 0; y < G; ++y) x[y] = (y < ng) ? d.lvl2[(size_t)y * b.nv + v] : 0.0;
  double s = 0.0;
#pragma unroll
  for (int y = 0; y < G; ++y) s += x[y];
  batch_store<KP>(b, d, v, s);
}

template <int KP>
__global__ void __launch_bounds__(64) batch_finalize2_kernel(BatchArgs b) {
  batch_finalize2_run<KP>(b, blockIdx.x, blockIdx.y, threadIdx.x);
}

// line search of graph gi (a 256-thread workgroup)
template <int KP>
__device__ inline void batch_linesearch_run(const BatchArgs& b, int gi, double alpha0,
                                            int first_fixed) {
  const BatchGraph& d = b.graphs[gi];
  if (*d.active == 0) return;
  linesearch_body<KP>(b.variant, first_fixed, alpha0, d.sc, d.status, nullptr, false,
                      b.freeze_eps, (b.upper != 0 && d.upk != nullptr) ? 1 : 0);
}

template <int KP>
__global__ void __launch_bounds__(256) batch_linesearch_kernel(BatchArgs b, double alpha0,
                                                               int first_fixed) {
  // the group's step counter: this is the last pass that reads the step's
  // scalars, and the residual of the next step reads the new value
  if (blockIdx.x == 0 && threadIdx.x == 0) *b.tcount += 1;
  batch_linesearch_run<KP>(b, blockIdx.x, alpha0, first_fixed);
}

// residual of X^t of graph gi (a 256-thread workgroup); a graph whose
// residual meets the tolerance (or whose status turned non-zero) stops
// iterating with this X
template <int KP>
__device__ inline void batch_residual_run(const BatchArgs& b, int gi) {
  const BatchGraph& d = b.graphs[gi];
  if (*d.active == 0) return;
  residual_body<KP>(b.variant, d.normA2, d.sc, d.status, 0.0, nullptr);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double rr = d.sc[SC<KP>::RELRES];
    const int64_t t = *b.tcount;  // the step index, kept on the device (graph replays)
    if ((b.tol > 0.0 && rr <= b.tol) || *d.status != 0) {
      *d.active = 0;
      *d.done_iter = t;
    } else if (b.tol > 0.0) {
      // stall test: less than 5% decrease over the last kBatchHist checks
      const int64_t c = t / b.check_every;
      const int slot = (int)(c % kBatchHist);
      const double old = d.hist[slot];
      if (c >= kBatchHist && rr > 0.95 * old) {
        *d.active = 0;
        *d.stalled = 1;
      }
      d.hist[slot] = rr;
    }
  }
}

template <int KP>
__global__ void __launch_bounds__(256) batch_residual_kernel(BatchArgs b) {
  batch_residual_run<KP>(b, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Persistent form of the batched lockstep loop (f1 and TriOFM-f1, FP32, two
// products with A per update): one cooperative launch per width group runs a
// chunk of updates, the passes of the per-pass launches one after another
// with a grid-wide barrier between them (every pass ends in a per-graph
// reduction that the next pass reads).  Workgroup blk does what workgroup blk
// of a per-pass launch with the same number of workers does, so the results
// are bitwise those of the per-pass launches; the 64-lane reductions are
// dealt to the waves, the line searches and residuals to the workgroups.
// ---------------------------------------------------------------------------

// Sense-reversing barrier over the nblk workgroups of a cooperative launch
// (bar[0]: arrivals, bar[1]: generation).  The agent-scope release / acquire
// fences make each workgroup's global writes visible to every XCD.  A wait
// longer than kBarrierSpins polls sets *err and lets the workgroup go on
// (then every later barrier of the launch is skipped), so the kernel always
// ends; the host reports the flag as an error.
constexpr long kBarrierSpins = 1L << 24;
__device__ inline void grid_barrier(unsigned* bar, int* err, unsigned nblk) {
  // every wave's stores have reached its XCD's L2 before the release below
  // writes the dirty lines back
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned arrived =
          __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == nblk - 1) {
        __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(bar + 1, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        long spins = 0;
        while (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          __builtin_amdgcn_s_sleep(1);
          if (++spins > kBarrierSpins) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// the per-graph reduction of a pass: first level, then (more than kFinChunk
// workers) the second, each 64-lane block of the per-pass grid taken by a wave
template <int KP>
__device__ inline void persist_finalize(const BatchArgs& b, unsigned* bar, int* err) {
  constexpr int WPB = Cfg<float, KP>::WPB;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * WPB + (threadIdx.x >> 6);
  const int nwv = gridDim.x * WPB;
  const int nx = (b.nv + 63) / 64;
  const int groups = (b.workers + kFinChunk - 1) / kFinChunk;
  const int n1 = nx * b.ngraphs * groups;
  for (int q = gw; q < n1; q += nwv)
    batch_finalize_run<KP>(b, q % nx, (q / nx) % b.ngraphs, q / (nx * b.ngraphs), lane);
  grid_barrier(bar, err, gridDim.x);
  if (groups > 1) {
    for (int q = gw; q < nx * b.ngraphs; q += nwv)
      batch_finalize2_run<KP>(b, q % nx, q / nx, lane);
    grid_barrier(bar, err, gridDim.x);
  }
}

// Compiled for two waves per SIMD (two workgroups per CU): with every pass
// inlined the compiler would otherwise take the whole register file, one wave
// per SIMD, too few gathers in flight for the products with A.
template <int KP>
__global__ void __launch_bounds__((Cfg<float, KP>::WPB * 64), 2)
    batch_persist_kernel(BatchPersistArgs p) {
  static_assert(Cfg<float, KP>::WPB * 64 == 256, "the line search and residual need 256 threads");
  extern __shared__ __align__(16) unsigned char smem[];
  for (int s = 0; s < p.steps; ++s) {
    const int64_t t = p.t0 + s;
    const int cur = p.cur0 ^ (s & 1);
    const bool check = (t % p.pass[kPGF1][0].check_every) == 0;
    {
      const BatchArgs& b = p.pass[check ? kPGF1C : kPGF1][cur];
      if (check) batch_spmm_run<KP, kGF1, true, false>(b, blockIdx.x, smem);
      else batch_spmm_run<KP, kGF1, false, false>(b, blockIdx.x, smem);
      grid_barrier(p.bar, p.err, gridDim.x);
      persist_finalize<KP>(b, p.bar, p.err);
      if (check) {
        for (int gi = blockIdx.x; gi < b.ngraphs; gi += gridDim.x) {
          batch_residual_run<KP>(b, gi);
          __syncthreads();
        }
        grid_barrier(p.bar, p.err, gridDim.x);
      }
    }
    {
      const BatchArgs& b = p.pass[kPVPass][cur];
      batch_dense_run<KP, kVPass>(b, blockIdx.x, smem);
      grid_barrier(p.bar, p.err, gridDim.x);
      persist_finalize<KP>(b, p.bar, p.err);
    }
    {
      const BatchArgs& b = p.pass[kPAV][cur];
      batch_spmm_run<KP, kAVF1, false, false>(b, blockIdx.x, smem);
      grid_barrier(p.bar, p.err, gridDim.x);
      persist_finalize<KP>(b, p.bar, p.err);
      // the step counter is read by the residual of the next step only
      if (blockIdx.x == 0 && threadIdx.x == 0) *b.tcount += 1;
      for (int gi = blockIdx.x; gi < b.ngraphs; gi += gridDim.x) {
        batch_linesearch_run<KP>(b, gi, p.alpha0, 0);
        __syncthreads();
      }
      grid_barrier(p.bar, p.err, gridDim.x);
    }
    {
      const BatchArgs& b = p.pass[kPUpdate][cur];
      batch_dense_run<KP, kUpdate>(b, blockIdx.x, smem);
      grid_barrier(p.bar, p.err, gridDim.x);
      persist_finalize<KP>(b, p.bar, p.err);
    }
  }
}

template <int KP>
static int persist_smem() {
  int m = Smem<float, KP, kGF1>::bytes;
  m = m > Smem<float, KP, kVPass>::bytes ? m : Smem<float, KP, kVPass>::bytes;
  m = m > Smem<float, KP, kAVF1>::bytes ? m : Smem<float, KP, kAVF1>::bytes;
  m = m > Smem<float, KP, kUpdate>::bytes ? m : Smem<float, KP, kUpdate>::bytes;
  return m;
}

template <int KP>
static hipError_t persist_launch_t(BatchPersistArgs& p, int max_workers, int* used_workers,
                                   hipStream_t s) {
  const int smem = persist_smem<KP>();
  int occ = 0, dev = 0, cus = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_persist_kernel<KP>,
                                                              256, smem);
  if (e != hipSuccess) return e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  // every workgroup must be resident at once (the barriers wait for all)
  int workers = (occ * cus) / 8;
  if (workers > max_workers) workers = max_workers;
  if (workers < 1) return hipErrorCooperativeLaunchTooLarge;
  for (auto& row : p.pass)
    for (auto& a : row) a.workers = workers;
  *used_workers = workers;
  void* args[] = {&p};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batch_persist_kernel<KP>),
                                    dim3(8 * workers), dim3(256), args, smem, s);
}

hipError_t launch_batch_persist(int k, BatchPersistArgs& p, int max_workers, int* used_workers,
                                hipStream_t s) {
  switch (k) {
    case 4: return persist_launch_t<4>(p, max_workers, used_workers, s);
    case 8: return persist_launch_t<8>(p, max_workers, used_workers, s);
    case 16: return persist_launch_t<16>(p, max_workers, used_workers, s);
    case 32: return persist_launch_t<32>(p, max_workers, used_workers, s);
  }
  return hipErrorInvalidValue;
}

// A batched pass runs 8 x workers workgroups; workers is trimmed so that the
// whole grid is resident at once (the per-graph loops give workgroups unequal
// work, so a second round would mostly run at low occupancy).  The reduction
// of the pass reads b.workers, so it sees the trimmed value.
template <auto Kernel>
static hipError_t launch_batch(BatchArgs& b, int threads, int smem, hipStream_t s) {
  const int cap = resident_blocks<Kernel>(threads, smem);
  if (cap >= 8 && b.workers > cap / 8) b.workers = cap / 8;
  hipLaunchKernelGGL(Kernel, dim3(8 * b.workers), dim3(threads), smem, s, b);
  return hipGetLastError();
}

template <int KP>
static hipError_t batch_spmm_t(BatchArgs& b, hipStream_t s) {
  const bool chk = (b.flags & kFlagCheck) != 0;
#define OFM_BSPMM(MODE)                                                                         \
  {                                                                                             \
    using SM = Smem<float, KP, MODE>;                                                           \
    constexpr int T = SM::WPB * 64;                                                             \
    if (b.bf16)                                                                                 \
      return chk ? launch_batch<batch_spmm_kernel<KP, MODE, true, true>>(b, T, SM::bytes, s)   \
                 : launch_batch<batch_spmm_kernel<KP, MODE, false, true>>(b, T, SM::bytes, s); \
    return chk ? launch_batch<batch_spmm_kernel<KP, MODE, true, false>>(b, T, SM::bytes, s)    \
               : launch_batch<batch_spmm_kernel<KP, MODE, false, false>>(b, T, SM::bytes, s);  \
  }
  switch (b.mode) {
    case kGF1: OFM_BSPMM(kGF1)
    case kAXF2: OFM_BSPMM(kAXF2)
    case kAVF1: OFM_BSPMM(kAVF1)
    case kAVF2: OFM_BSPMM(kAVF2)
  }
#undef OFM_BSPMM
  return hipErrorInvalidValue;
}

template <int KP>
static hipError_t batch_dense_t(BatchArgs& b, hipStream_t s) {
#define OFM_BDENSE(MODE)                                                                  \
  {                                                                                       \
    using SM = Smem<float, KP, MODE>;                                                     \
    return launch_batch<batch_dense_kernel<KP, MODE>>(b, SM::WPB * 64, SM::bytes, s);    \
  }
  switch (b.mode) {
    case kGPassF2: OFM_BDENSE(kGPassF2)
    case kGPassF1: OFM_BDENSE(kGPassF1)
    case kVPass: OFM_BDENSE(kVPass)
    case kUpdate: OFM_BDENSE(kUpdate)
    case kUpdateR: OFM_BDENSE(kUpdateR)
    case kGramM: OFM_BDENSE(kGramM)
  }
#undef OFM_BDENSE
  return hipErrorInvalidValue;
}

int batch_wpb(int k) { return wpb(OFM_FP32, k); }

hipError_t launch_batch_spmm(int k, BatchArgs& b, hipStream_t s) {
  switch (k) {
    case 4: return batch_spmm_t<4>(b, s);
    case 8: return batch_spmm_t<8>(b, s);
    case 16: return batch_spmm_t<16>(b, s);
    case 32: return batch_spmm_t<32>(b, s);
    case 64: return batch_spmm_t<64>(b, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_dense(int k, BatchArgs& b, hipStream_t s) {
  switch (k) {
    case 4: return batch_dense_t<4>(b, s);
    case 8: return batch_dense_t<8>(b, s);
    case 16: return batch_dense_t<16>(b, s);
    case 32: return batch_dense_t<32>(b, s);
    case 64: return batch_dense_t<64>(b, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_batch_finalize(BatchArgs& b, hipStream_t s) {
  if (b.nv == 0) return hipSuccess;
  const int groups = (b.workers + kFinChunk - 1) / kFinChunk;
  const dim3 grid((b.nv + 63) / 64, b.ngraphs, groups);
  const dim3 grid2((b.nv + 63) / 64, b.ngraphs);
#define OFM_BFIN(KP)                                                                        \
  hipLaunchKernelGGL(batch_finalize_kernel<KP>, grid, dim3(64), 0, s, b);                  \
  if (groups > 1) hipLaunchKernelGGL(batch_finalize2_kernel<KP>, grid2, dim3(64), 0, s, b); \
  break;
  switch (b.k) {
    case 4: OFM_BFIN(4)
    case 8: OFM_BFIN(8)
    case 16: OFM_BFIN(16)
    case 32: OFM_BFIN(32)
    case 64: OFM_BFIN(64)
    default: return hipErrorInvalidValue;
  }
#undef OFM_BFIN
  return hipGetLastError();
}

hipError_t launch_batch_linesearch(int k, BatchArgs& b, double alpha0, int first_fixed,
                                   hipStream_t s) {
  switch (k) {
    case 4: hipLaunchKernelGGL(batch_linesearch_kernel<4>, dim3(b.ngraphs), dim3(256), 0, s, b, alpha0, first_fixed); break;
    case 8: hipLaunchKernelGGL(batch_linesearch_kernel<8>, dim3(b.ngraphs), dim3(256), 0, s, b, alpha0, first_fixed); break;
    case 16: hipLaunchKernelGGL(batch_linesearch_kernel<16>, dim3(b.ngraphs), dim3(256), 0, s, b, alpha0, first_fixed); break;
    case 32: hipLaunchKernelGGL(batch_linesearch_kernel<32>, dim3(b.ngraphs), dim3(256), 0, s, b, alpha0, first_fixed); break;
    case 64: hipLaunchKernelGGL(batch_linesearch_kernel<64>, dim3(b.ngraphs), dim3(256), 0, s, b, alpha0, first_fixed); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_residual(int k, BatchArgs& b, hipStream_t s) {
  switch (k) {
    case 4: hipLaunchKernelGGL(batch_residual_kernel<4>, dim3(b.ngraphs), dim3(256), 0, s, b); break;
    case 8: hipLaunchKernelGGL(batch_residual_kernel<8>, dim3(b.ngraphs), dim3(256), 0, s, b); break;
    case 16: hipLaunchKernelGGL(batch_residual_kernel<16>, dim3(b.ngraphs), dim3(256), 0, s, b); break;
    case 32: hipLaunchKernelGGL(batch_residual_kernel<32>, dim3(b.ngraphs), dim3(256), 0, s, b); break;
    case 64: hipLaunchKernelGGL(batch_residual_kernel<64>, dim3(b.ngraphs), dim3(256), 0, s, b); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ofm
