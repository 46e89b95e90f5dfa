// Post-processing of Algorithm 1 (steps 4-5): row normalisation and
// Euclidean K-means (assignment, deterministic centroid update, k-means++
// seeding from caller-supplied uniforms).
#include <math.h>
#include <stdint.h>

#include "ofm_internal.hpp"

namespace ofm {

// Row-wise kernels: a group of kRowLanes lanes per row, element c of the row
// in lane c % kRowLanes (k <= 64, so at most 4 elements per lane); grid-stride
// over the rows.
constexpr int kRowLanes = 16;

__device__ inline double group_sum(double x) {
#pragma unroll
  for (int o = kRowLanes / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, kRowLanes);
  return __shfl(x, 0, kRowLanes);  // every lane takes lane 0's sum
}

__device__ inline float group_sum(float x) {
#pragma unroll
  for (int o = kRowLanes / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, kRowLanes);
  return __shfl(x, 0, kRowLanes);
}

static unsigned row_blocks(int64_t n) {
  const int64_t groups_per_block = 256 / kRowLanes;
  int64_t nb = (n + groups_per_block - 1) / groups_per_block;
  if (nb > 4096) nb = 4096;
  return (unsigned)(nb < 1 ? 1 : nb);
}

// X and Y may be the same block: each element is read before it is written,
// by the same lane, so neither pointer is restrict-qualified.
template <typename T>
__global__ void __launch_bounds__(256) row_normalize_kernel(int64_t n, int k, const T* X, T* Y) {
  const int lane = threadIdx.x % kRowLanes;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kRowLanes; i < n;
       i += stride) {
    T v[4];
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = lane + q * kRowLanes;
      v[q] = c < k ? X[i * k + c] : T(0);
      s += (double)v[q] * (double)v[q];
    }
    const double nr = sqrt(group_sum(s));
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = lane + q * kRowLanes;
      if (c < k) Y[i * k + c] = nr > 0.0 ? (T)((double)v[q] / nr) : T(0);
    }
  }
}

// Rows whose byte length is 16 L with L a power of two (k = 32 in FP32: L = 8):
// the block is a flat array of 16-byte vectors, lane t takes vector t, and the
// L lanes of one row sum their squares with a width-L butterfly.  Loads and
// stores are then 16 bytes per lane and contiguous across the wavefront.
template <int W>
__device__ inline double width_sum(double x) {
#pragma unroll
  for (int o = W / 2; o >= 1; o >>= 1) x += __shfl_xor(x, o, W);
  return x;
}

template <typename T, int L>
__global__ void __launch_bounds__(256) row_normalize_vec_kernel(int64_t n, const T* X, T* Y) {
  constexpr int E = 16 / sizeof(T);
  typedef T vec __attribute__((ext_vector_type(E)));
  const int64_t total = n * L;  // vectors; the L of one row share a loop trip
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
    vec v = reinterpret_cast<const vec*>(X)[t];
    double sq = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) sq += (double)v[e] * (double)v[e];
    const double nr = sqrt(width_sum<L>(sq));
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = nr > 0.0 ? (T)((double)v[e] / nr) : T(0);
    reinterpret_cast<vec*>(Y)[t] = v;
  }
}

template <typename T, int L>
static hipError_t row_normalize_vec(int64_t n, const void* X, void* Y, hipStream_t s) {
  int64_t nb = (n * L + 255) / 256;
  if (nb > 2048) nb = 2048;  // one resident round (8 blocks per CU)
  hipLaunchKernelGGL((row_normalize_vec_kernel<T, L>), dim3((unsigned)nb), dim3(256), 0, s, n,
                     static_cast<const T*>(X), static_cast<T*>(Y));
  return hipGetLastError();
}

template <typename T>
static hipError_t row_normalize_vec_any(int64_t n, int L, const void* X, void* Y, hipStream_t s) {
  switch (L) {
    case 1: return row_normalize_vec<T, 1>(n, X, Y, s);
    case 2: return row_normalize_vec<T, 2>(n, X, Y, s);
    case 4: return row_normalize_vec<T, 4>(n, X, Y, s);
    case 8: return row_normalize_vec<T, 8>(n, X, Y, s);
    case 16: return row_normalize_vec<T, 16>(n, X, Y, s);
    default: return row_normalize_vec<T, 32>(n, X, Y, s);  // k = 64 in FP64
  }
}

hipError_t launch_row_normalize(int64_t n, int k, int precision, const void* X, void* Y,
                                hipStream_t s) {
  const int esz = precision == OFM_FP64 ? 8 : 4;
  const int rb = k * esz;
  const int L = rb / 16;
  if (rb % 16 == 0 && L >= 1 && L <= 32 && (L & (L - 1)) == 0 &&
      reinterpret_cast<uintptr_t>(X) % 16 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0)
    return precision == OFM_FP64 ? row_normalize_vec_any<double>(n, L, X, Y, s)
                                 : row_normalize_vec_any<float>(n, L, X, Y, s);
  const unsigned nb = row_blocks(n);
  if (precision == OFM_FP64)
    hipLaunchKernelGGL(row_normalize_kernel<double>, dim3(nb), dim3(256), 0, s, n, k,
                       static_cast<const double*>(X), static_cast<double*>(Y));
  else
    hipLaunchKernelGGL(row_normalize_kernel<float>, dim3(nb), dim3(256), 0, s, n, k,
                       static_cast<const float*>(X), static_cast<float*>(Y));
  return hipGetLastError();
}

// Y = s[0] * X elementwise (s: one FP64 in device memory)
template <typename T>
__global__ void __launch_bounds__(256) scale_kernel(int64_t count, const double* __restrict__ sp,
                                                    const T* X, T* Y) {
  const double sc = sp[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    Y[i] = (T)(sc * (double)X[i]);
}

hipError_t launch_scale(int64_t count, int precision, const double* sp, const void* X, void* Y,
                        hipStream_t s) {
  int64_t nb = (count + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (precision == OFM_FP64)
    hipLaunchKernelGGL(scale_kernel<double>, dim3((unsigned)nb), dim3(256), 0, s, count, sp,
                       static_cast<const double*>(X), static_cast<double*>(Y));
  else
    hipLaunchKernelGGL(scale_kernel<float>, dim3((unsigned)nb), dim3(256), 0, s, count, sp,
                       static_cast<const float*>(X), static_cast<float*>(Y));
  return hipGetLastError();
}

__global__ void convert_kernel(int64_t count, int to_fp64, const void* __restrict__ src,
                               void* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  if (to_fp64) static_cast<double*>(dst)[i] = (double)static_cast<const float*>(src)[i];
  else static_cast<float*>(dst)[i] = (float)static_cast<const double*>(src)[i];
}

hipError_t launch_convert(int64_t count, int to_fp64, const void* src, void* dst, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count,
                     to_fp64, src, dst);
  return hipGetLastError();
}

// One point per thread: the row sits in registers (padded with zeros to D),
// the centroids are read from LDS with every lane at the same address (a
// broadcast), padded with zeros to D as well, so the padding adds nothing to
// the distances.  When all centroids do not fit in kAssignLdsFloats they are
// staged chunk by chunk for each tile of rows.
constexpr int kAssignLdsFloats = 8192;  // 32 KB of centroids per block
constexpr int kAssignThreads = 256;

template <int D>
__device__ inline void stage_centroids(float* cs, const float* __restrict__ C, int dim, int c0,
                                       int cn) {
  for (int e = threadIdx.x; e < cn * D; e += kAssignThreads) {
    const int c = e / D, d = e % D;
    cs[e] = d < dim ? C[(int64_t)(c0 + c) * dim + d] : 0.0f;
  }
}

// label_i = argmin_c sum_d (y_id - mu_cd)^2 (lowest c on ties), FP32 distances
template <int D>
__global__ void __launch_bounds__(kAssignThreads) kmeans_assign_kernel(
    int64_t n, int dim, int nc, const float* __restrict__ Y, const float* __restrict__ C,
    int32_t* __restrict__ labels, float* __restrict__ dist2, int chunk, int vec4) {
  extern __shared__ float cs[];
  const bool once = chunk >= nc;
  if (once) {
    stage_centroids<D>(cs, C, dim, 0, nc);
    __syncthreads();
  }
  // the tile loop is uniform over the block so that the chunked path can
  // synchronize inside it
  for (int64_t base = (int64_t)blockIdx.x * kAssignThreads; base < n;
       base += (int64_t)gridDim.x * kAssignThreads) {
    const int64_t i = base + threadIdx.x;
    float y[D];
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = 0.0f;
    if (i < n) {
      const float* row = Y + i * dim;
      if (vec4) {
#pragma unroll
        for (int q = 0; q < D / 4; ++q)
          if (4 * q < dim) {
            const float4 v = reinterpret_cast<const float4*>(row)[q];
            y[4 * q] = v.x;
            y[4 * q + 1] = v.y;
            y[4 * q + 2] = v.z;
            y[4 * q + 3] = v.w;
          }
      } else {
#pragma unroll
        for (int d = 0; d < D; ++d)
          if (d < dim) y[d] = row[d];
      }
    }
    float best = INFINITY;
    int bi = 0;
    for (int c0 = 0; c0 < nc; c0 += chunk) {
      const int cn = min(chunk, nc - c0);
      if (!once) {
        __syncthreads();
        stage_centroids<D>(cs, C, dim, c0, cn);
        __syncthreads();
      }
      for (int c = 0; c < cn; ++c) {
        const float4* mu = reinterpret_cast<const float4*>(cs + c * D);
        float sq = 0.0f;
#pragma unroll
        for (int q = 0; q < D / 4; ++q) {
          const float4 m = mu[q];
          float t = y[4 * q] - m.x;
          sq = fmaf(t, t, sq);
          t = y[4 * q + 1] - m.y;
          sq = fmaf(t, t, sq);
          t = y[4 * q + 2] - m.z;
          sq = fmaf(t, t, sq);
          t = y[4 * q + 3] - m.w;
          sq = fmaf(t, t, sq);
        }
        if (sq < best) {
          best = sq;
          bi = c0 + c;
        }
      }
    }
    if (i < n) {
      labels[i] = bi;
      if (dist2) dist2[i] = best;
    }
  }
}

template <int D>
static hipError_t assign_with(int64_t n, int dim, int nc, const float* Y, const float* C,
                              int32_t* labels, float* dist2, hipStream_t s) {
  const int chunk = nc * D <= kAssignLdsFloats ? nc : kAssignLdsFloats / D;
  const size_t smem = (size_t)chunk * D * sizeof(float);
  const int vec4 = (dim % 4 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0) ? 1 : 0;
  // one resident round of blocks (the tile loop strides over the rest), so no
  // partial last round leaves CUs idle; the LDS size depends on the call
  int occ = 0, dev = 0, cus = 0;
  int64_t cap = 2048;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kmeans_assign_kernel<D>, kAssignThreads,
                                                   smem) == hipSuccess &&
      hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      occ > 0 && cus > 0)
    cap = (int64_t)occ * cus;
  int64_t nb = (n + kAssignThreads - 1) / kAssignThreads;
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(kmeans_assign_kernel<D>, dim3((unsigned)nb), dim3(kAssignThreads), smem, s,
                     n, dim, nc, Y, C, labels, dist2, chunk, vec4);
  return hipGetLastError();
}

hipError_t launch_kmeans_assign(int64_t n, int dim, int nc, const float* Y, const float* C,
                                int32_t* labels, float* dist2, hipStream_t s) {
  if (dim <= 4) return assign_with<4>(n, dim, nc, Y, C, labels, dist2, s);
  if (dim <= 8) return assign_with<8>(n, dim, nc, Y, C, labels, dist2, s);
  if (dim <= 16) return assign_with<16>(n, dim, nc, Y, C, labels, dist2, s);
  if (dim <= 32) return assign_with<32>(n, dim, nc, Y, C, labels, dist2, s);
  return assign_with<64>(n, dim, nc, Y, C, labels, dist2, s);
}

// ---------------------------------------------------------------------------
// Lloyd centroid update: per-block sums of the rows of every cluster plus
// counts, then means.  Every sum has a fixed order (rows in order within a
// wave, waves and blocks in order), so the result does not depend on timing.
// part layout: [block][nc][dim + 1].
// ---------------------------------------------------------------------------
constexpr int kSumWaves = 4;
constexpr int kSumRows = 16;           // rows whose loads a wave keeps in flight
constexpr int kSumLdsDoubles = 2048;   // per wave: nc (dim + 1) <= 2048 takes the LDS path
constexpr int64_t kPartBytes = int64_t(256) << 20;

int kmeans_blocks(int64_t n, int nv) {
  int64_t nb = (n + 2047) / 2048;
  if (nb > 1024) nb = 1024;
  const int64_t cap = kPartBytes / ((int64_t)nv * (int64_t)sizeof(double));
  if (nb > cap) nb = cap;
  if (nb < 1) nb = 1;
  return (int)nb;
}

// kSumWaves waves per block, each over a contiguous quarter of the block's
// rows with its own LDS accumulator (lane = feature); the quarters are added
// in wave order at the end.
__global__ void __launch_bounds__(kSumWaves * 64) kmeans_sums_lds_kernel(
    int64_t n, int dim, int nc, const float* __restrict__ Y, const int32_t* __restrict__ labels,
    double* __restrict__ part) {
  extern __shared__ double acc[];
  const int nv = nc * (dim + 1);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e = threadIdx.x; e < kSumWaves * nv; e += blockDim.x) acc[e] = 0.0;
  __syncthreads();
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = min(n, r0 + per);
  const int64_t len = r1 > r0 ? r1 - r0 : 0;
  const int64_t w0 = r0 + len * w / kSumWaves, w1 = r0 + len * (w + 1) / kSumWaves;
  double* a = acc + (size_t)w * nv;
  // the loads of a batch are unconditional (row and feature clamped into
  // range, the value masked afterwards) so that all of them are in flight
  // together
  const int f = lane < dim ? lane : dim - 1;
  for (int64_t rb = w0; rb < w1; rb += kSumRows) {
    int lab[kSumRows];
    float y[kSumRows];
#pragma unroll
    for (int q = 0; q < kSumRows; ++q) {
      const int64_t r = rb + q < w1 ? rb + q : w1 - 1;
      lab[q] = labels[r];
      y[q] = Y[r * dim + f];
    }
#pragma unroll
    for (int q = 0; q < kSumRows; ++q) {
      if (rb + q >= w1) lab[q] = -1;
      if (lane >= dim) y[q] = 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kSumRows; ++q) {
      if (lab[q] >= 0) {
        double* ac = a + (size_t)lab[q] * (dim + 1);
        if (lane < dim) ac[lane] += (double)y[q];
        if (lane == 0) ac[dim] += 1.0;
      }
    }
  }
  __syncthreads();
  double* pb = part + (size_t)blockIdx.x * nv;
  for (int e = threadIdx.x; e < nv; e += blockDim.x) {
    double t = acc[e];
    for (int v = 1; v < kSumWaves; ++v) t += acc[(size_t)v * nv + e];
    pb[e] = t;
  }
}

// many clusters: one wave per block accumulating into its own partial row
__global__ void __launch_bounds__(64) kmeans_sums_global_kernel(int64_t n, int dim, int nc,
                                                                const float* __restrict__ Y,
                                                                const int32_t* __restrict__ labels,
                                                                double* __restrict__ part) {
  const int lane = threadIdx.x;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = min(n, r0 + per);
  const int nv = nc * (dim + 1);
  double* acc = part + (size_t)blockIdx.x * nv;
  for (int e = lane; e < nv; e += 64) acc[e] = 0.0;
  __syncthreads();  // zeroed by other lanes than those that accumulate
  for (int64_t r = r0; r < r1; ++r) {
    const int c = labels[r];
    if (lane < dim) acc[(size_t)c * (dim + 1) + lane] += (double)Y[r * dim + lane];
    if (lane == 0) acc[(size_t)c * (dim + 1) + dim] += 1.0;
  }
}

// centroid c = (sum of its rows) / count, or the old centroid when empty;
// block c, lane = feature (two rounds for dim + 1 > 64), wave v sums the
// blocks v, v + 4, ... in order, the four waves are added in order.
__global__ void __launch_bounds__(kSumWaves * 64) kmeans_final_kernel(
    int dim, int nc, const double* __restrict__ part, int nb, const float* __restrict__ old_c,
    float* __restrict__ new_c) {
  __shared__ double red[kSumWaves][2][64];
  const int c = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nv = nc * (dim + 1);
  constexpr int kB = 8;  // partial rows whose loads are in flight together
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int d = h * 64 + lane;
    const int dc = d <= dim ? d : dim;
    double s = 0.0;
    for (int b0 = w; b0 < nb; b0 += kB * kSumWaves) {
      double x[kB];
#pragma unroll
      for (int q = 0; q < kB; ++q) {
        const int b = b0 + q * kSumWaves;
        x[q] = part[(size_t)(b < nb ? b : nb - 1) * nv + (size_t)c * (dim + 1) + dc];
      }
#pragma unroll
      for (int q = 0; q < kB; ++q)
        if (b0 + q * kSumWaves < nb) s += x[q];
    }
    red[w][h][lane] = d <= dim ? s : 0.0;
  }
  __syncthreads();
  if (w != 0) return;
  double cnt = 0.0;
  {
    const int hc = dim / 64, lc = dim % 64;
    for (int v = 0; v < kSumWaves; ++v) cnt += red[v][hc][lc];
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int d = h * 64 + lane;
    if (d < dim) {
      double t = 0.0;
      for (int v = 0; v < kSumWaves; ++v) t += red[v][h][lane];
      new_c[(size_t)c * dim + d] = cnt > 0.0 ? (float)(t / cnt) : old_c[(size_t)c * dim + d];
    }
  }
}

hipError_t launch_kmeans_centroid_sums(int64_t n, int dim, int nc, const float* Y,
                                       const int32_t* labels, double* part, int nb,
                                       hipStream_t s) {
  const int nv = nc * (dim + 1);
  if (nv <= kSumLdsDoubles)
    hipLaunchKernelGGL(kmeans_sums_lds_kernel, dim3(nb), dim3(kSumWaves * 64),
                       (size_t)kSumWaves * nv * sizeof(double), s, n, dim, nc, Y, labels, part);
  else
    hipLaunchKernelGGL(kmeans_sums_global_kernel, dim3(nb), dim3(64), 0, s, n, dim, nc, Y, labels,
                       part);
  return hipGetLastError();
}

hipError_t launch_kmeans_centroid_final(int dim, int nc, const double* part, int nb,
                                        const float* old_c, float* new_c, hipStream_t s) {
  hipLaunchKernelGGL(kmeans_final_kernel, dim3(nc), dim3(kSumWaves * 64), 0, s, dim, nc, part, nb,
                     old_c, new_c);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-means++ seeding.  The points are cut into nb chunks of `per` rows.  A
// chunk's running sums of D^2 (FP64) are formed in rounds of 256 rows with a
// block-wide inclusive scan; the distance kernel stores the chunk totals, and
// the pick kernel repeats the same rounds on the chosen chunk only, so both
// see bitwise the same running sums.
// ---------------------------------------------------------------------------
constexpr int kScan = 256;
constexpr int kPickChunks = 1024;

int kmeans_pick_chunks(int64_t n) { return (int)(n < kPickChunks ? n : kPickChunks); }

// inclusive scan of one value per thread over the block, fixed order
__device__ inline double block_scan(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < kScan; o <<= 1) {
    const double add = t >= o ? sh[t - o] : 0.0;
    __syncthreads();
    v += add;
    sh[t] = v;
    __syncthreads();
  }
  return v;
}

// d2[i] = min(d2[i], ||y_i - centre||^2) (first: the distance itself), and
// the chunk totals of d2 in sums[chunk]
__global__ void __launch_bounds__(kScan) kmeans_mindist_kernel(int64_t n, int dim,
                                                               const float* __restrict__ Y,
                                                               const float* __restrict__ centre,
                                                               float* __restrict__ d2, int first,
                                                               int64_t per, int vec4,
                                                               double* __restrict__ sums) {
  __shared__ double sh[kScan];
  __shared__ float cs[64];
  if (threadIdx.x < dim) cs[threadIdx.x] = centre[threadIdx.x];
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = min(n, r0 + per);
  double carry = 0.0;
  for (int64_t base = r0; base < r1; base += kScan) {
    const int64_t r = base + threadIdx.x;
    double v = 0.0;
    if (r < r1) {
      float sq = 0.0f;
      if (vec4) {
        const float4* row = reinterpret_cast<const float4*>(Y + r * dim);
        for (int q = 0; q < dim / 4; ++q) {
          const float4 y = row[q];
          float t = y.x - cs[4 * q];
          sq = fmaf(t, t, sq);
          t = y.y - cs[4 * q + 1];
          sq = fmaf(t, t, sq);
          t = y.z - cs[4 * q + 2];
          sq = fmaf(t, t, sq);
          t = y.w - cs[4 * q + 3];
          sq = fmaf(t, t, sq);
        }
      } else {
        for (int d = 0; d < dim; ++d) {
          const float t = Y[r * dim + d] - cs[d];
          sq = fmaf(t, t, sq);
        }
      }
      const float nd = first ? sq : fminf(d2[r], sq);
      d2[r] = nd;
      v = (double)nd;
    }
    block_scan(v, sh);
    const int last = (int)min((int64_t)kScan - 1, r1 - 1 - base);
    carry += sh[last];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = carry;
}

hipError_t launch_kmeans_mindist(int64_t n, int dim, const float* Y, const float* centre,
                                 float* d2, int first, double* sums, hipStream_t s) {
  const int nb = kmeans_pick_chunks(n);
  const int64_t per = (n + nb - 1) / nb;
  const int vec4 = (dim % 4 == 0 && reinterpret_cast<uintptr_t>(Y) % 16 == 0) ? 1 : 0;
  hipLaunchKernelGGL(kmeans_mindist_kernel, dim3(nb), dim3(kScan), 0, s, n, dim, Y, centre, d2,
                     first, per, vec4, sums);
  return hipGetLastError();
}

// first point whose running sum of d2 exceeds u * total; the previous pick
// stays when the total is zero (every point sits on a chosen centre)
__global__ void __launch_bounds__(kScan) kmeans_pick_kernel(int64_t n, const float* __restrict__ d2,
                                                            const double* __restrict__ sums,
                                                            int nb, int64_t per, double u,
                                                            int32_t* pick) {
  __shared__ double sh[kScan];
  __shared__ double ex[kPickChunks];
  __shared__ int best_b;
  __shared__ unsigned long long best_r;
  const int t = threadIdx.x;
  // exclusive prefix sums of the chunk totals, rounds of 256 chunks
  double carry = 0.0;
  for (int base = 0; base < nb; base += kScan) {
    const int b = base + t;
    const double v = b < nb ? sums[b] : 0.0;
    block_scan(v, sh);
    if (b < nb) ex[b] = t == 0 ? carry : carry + sh[t - 1];
    const int last = min(kScan - 1, nb - 1 - base);
    carry += sh[last];
    __syncthreads();
  }
  const double tot = carry;
  if (!(tot > 0.0)) return;
  const double target = u * tot;
  if (t == 0) {
    best_b = nb;
    best_r = (unsigned long long)n;
  }
  __syncthreads();
  for (int b = t; b < nb; b += kScan)
    if (ex[b] + sums[b] > target) atomicMin(&best_b, b);
  __syncthreads();
  const int b = best_b;
  if (b >= nb) {
    if (t == 0) pick[0] = (int32_t)(n - 1);
    return;
  }
  // the same rounds as the distance kernel over chunk b
  const double exb = ex[b];
  const int64_t r0 = (int64_t)b * per;
  const int64_t r1 = min(n, r0 + per);
  double lc = 0.0;
  for (int64_t base = r0; base < r1; base += kScan) {
    const int64_t r = base + t;
    const double v = r < r1 ? (double)d2[r] : 0.0;
    const double incl = block_scan(v, sh);
    if (r < r1 && exb + (lc + incl) > target) atomicMin(&best_r, (unsigned long long)r);
    const int last = (int)min((int64_t)kScan - 1, r1 - 1 - base);
    lc += sh[last];
    __syncthreads();
    if (best_r < (unsigned long long)n) break;
  }
  if (t == 0) pick[0] = (int32_t)(best_r < (unsigned long long)n ? (int64_t)best_r : r1 - 1);
}

hipError_t launch_kmeans_pick(int64_t n, const float* d2, double u, const double* sums,
                              int32_t* pick, hipStream_t s) {
  const int nb = kmeans_pick_chunks(n);
  const int64_t per = (n + nb - 1) / nb;
  hipLaunchKernelGGL(kmeans_pick_kernel, dim3(1), dim3(kScan), 0, s, n, d2, sums, nb, per, u,
                     pick);
  return hipGetLastError();
}

__global__ void kmeans_copy_centre_kernel(int dim, const float* __restrict__ Y,
                                          const int32_t* __restrict__ pick, float* __restrict__ C,
                                          int c) {
  const int d = threadIdx.x;
  if (d < dim) C[(size_t)c * dim + d] = Y[(size_t)pick[0] * dim + d];
}

hipError_t launch_kmeans_copy_centre(int dim, const float* Y, const int32_t* pick, float* C, int c,
                                     hipStream_t s) {
  hipLaunchKernelGGL(kmeans_copy_centre_kernel, dim3(1), dim3(64), 0, s, dim, Y, pick, C, c);
  return hipGetLastError();
}

__global__ void count_changes_kernel(int64_t n, const int32_t* __restrict__ a,
                                     const int32_t* __restrict__ b, int* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int ch = (i < n && a[i] != b[i]) ? 1 : 0;
  // any change is enough: one atomic per block, not one per wavefront (many
  // atomics on one word serialize)
  if (__syncthreads_or(ch) && threadIdx.x == 0) atomicOr(out, 1);
}

hipError_t launch_count_changes(int64_t n, const int32_t* a, const int32_t* b, int* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(count_changes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                     a, b, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row-gather measurement: Y_r = sum of the S rows Z[idx[r S + e]], with rows of
// RF FP32 values read as 16-byte vectors by RF / 4 lanes (the access pattern of
// the products with A without their sparse-matrix bookkeeping).  A group of
// lanes per output row, CH gathers in flight per lane.
// ---------------------------------------------------------------------------

template <int RF, int CH>
__global__ void __launch_bounds__(256) gather_rows_kernel(int64_t nrows, int S,
                                                          const int32_t* __restrict__ idx,
                                                          const float4* __restrict__ Z,
                                                          float4* __restrict__ Y) {
  constexpr int L = RF / 4;        // lanes per row
  constexpr int G = 64 / L;        // rows per wave
  const int lane = threadIdx.x & 63, grp = lane / L, j = lane % L;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = wave * G + grp; r < nrows; r += nwaves * G) {
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const int32_t* ip = idx + r * S;
    for (int e0 = 0; e0 < S; e0 += CH) {
      int c[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) c[u] = (e0 + u < S) ? ip[e0 + u] : -1;
      float4 z[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u)
        z[u] = c[u] >= 0 ? Z[(int64_t)c[u] * L + j] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        acc.x += z[u].x;
        acc.y += z[u].y;
        acc.z += z[u].z;
        acc.w += z[u].w;
      }
    }
    Y[r * L + j] = acc;
  }
}

hipError_t launch_gather_rows(int64_t nrows, int S, int row_floats, const int32_t* idx,
                              const float* Z, float* Y, hipStream_t s) {
  const dim3 grid(8192), block(256);
  const float4* z = reinterpret_cast<const float4*>(Z);
  float4* y = reinterpret_cast<float4*>(Y);
  switch (row_floats) {
    case 16: hipLaunchKernelGGL((gather_rows_kernel<16, 16>), grid, block, 0, s, nrows, S, idx, z, y); break;
    case 32: hipLaunchKernelGGL((gather_rows_kernel<32, 16>), grid, block, 0, s, nrows, S, idx, z, y); break;
    case 64: hipLaunchKernelGGL((gather_rows_kernel<64, 16>), grid, block, 0, s, nrows, S, idx, z, y); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ofm
