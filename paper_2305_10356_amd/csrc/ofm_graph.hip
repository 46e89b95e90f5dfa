// Shifted normalized Laplacian set-up (Introduction, eq. (1); Algorithm 1,
// step 2):  D_ii = sum_j S_ij,  w_ij = D_ii^{-1/2} S_ij D_jj^{-1/2},
// A = -I - W.  Degrees, checks, weights and the packed (column, weight)
// stream in row-processing order are computed on the device.
#include <math.h>

#include "ofm_internal.hpp"

namespace ofm {

enum : int { kGraphBadPtr = 1, kGraphBadCol = 2, kGraphZeroDeg = 4, kGraphUnsorted = 8,
             kGraphAsym = 16, kGraphBadVal = 32 };

__global__ void graph_check_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ row_ptr,
                                   const int32_t* __restrict__ col_idx,
                                   const double* __restrict__ vals, double* __restrict__ deg,
                                   int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = row_ptr[i], e = row_ptr[i + 1];
  int f = 0;
  if (b < 0 || e < b || e > nnz) {
    atomicOr(flags, kGraphBadPtr);
    deg[i] = 0.0;
    return;
  }
  if (i == 0 && b != 0) f |= kGraphBadPtr;
  if (i == n - 1 && e != nnz) f |= kGraphBadPtr;
  double d = 0.0;
  int prev = -1;
  for (int64_t t = b; t < e; ++t) {
    const int c = col_idx[t];
    if (c < 0 || c >= n) f |= kGraphBadCol;
    if (c <= prev) f |= kGraphUnsorted;
    prev = c;
    const double v = vals ? vals[t] : 1.0;
    if (!(v >= 0.0) || !isfinite(v)) f |= kGraphBadVal;
    d += v;
  }
  if (!(d > 0.0)) f |= kGraphZeroDeg;
  deg[i] = d;
  if (f) atomicOr(flags, f);
}

// symmetric pattern (and weights): every stored (i, j) has a stored (j, i)
__global__ void graph_symcheck_kernel(int64_t n, const int32_t* __restrict__ row_ptr,
                                      const int32_t* __restrict__ col_idx,
                                      const double* __restrict__ vals, int sorted, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
    const int j = col_idx[t];
    int64_t lo = row_ptr[j], hi = row_ptr[j + 1];
    int64_t found = -1;
    if (sorted) {
      while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (col_idx[mid] < i) lo = mid + 1;
        else hi = mid;
      }
      if (lo < row_ptr[j + 1] && col_idx[lo] == i) found = lo;
    } else {
      for (int64_t u = lo; u < hi; ++u)
        if (col_idx[u] == i) {
          found = u;
          break;
        }
    }
    if (found < 0 || (vals && vals[found] != vals[t])) {
      atomicOr(flags, kGraphAsym);
      return;
    }
  }
}

// w_ij in CSR order, D^{-1/2}, and per-block partial sums of ||A||_F^2
// (row i contributes (1 + sum of its self-loop weights)^2 + sum_{j != i} w_ij^2)
__global__ void __launch_bounds__(256) graph_weights_kernel(int64_t n,
                                                            const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col_idx,
                                                            const double* __restrict__ vals,
                                                            const double* __restrict__ deg,
                                                            double* __restrict__ dinv,
                                                            double* __restrict__ w64,
                                                            double* __restrict__ part) {
  __shared__ double buf[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (i < n) {
    const double di = 1.0 / sqrt(deg[i]);
    dinv[i] = di;
    double self = 0.0, off = 0.0;
    for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
      const int j = col_idx[t];
      const double v = vals ? vals[t] : 1.0;
      const double w = di * v / sqrt(deg[j]);
      w64[t] = w;
      if (j == i) self += w;
      else off += w * w;
    }
    acc = (1.0 + self) * (1.0 + self) + off;
  }
  buf[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) buf[threadIdx.x] += buf[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = buf[0];
}

struct __align__(8) PkEnt32 {
  int col;
  float w;
};
struct __align__(16) PkEnt64 {
  int col;
  int pad;
  double w;
};

// entries of the row at position p, copied to the packed stream at sptr[p];
// a column whose row has fewer than cold_below entries (a rarely gathered row)
// is stored with its sign bit set, which the gathers mask off
__global__ void graph_pack_kernel(int64_t n, const int32_t* __restrict__ sched,
                                  const int32_t* __restrict__ row_ptr,
                                  const int32_t* __restrict__ col_idx,
                                  const double* __restrict__ w64,
                                  const int32_t* __restrict__ sptr, PkEnt32* __restrict__ pk32,
                                  PkEnt64* __restrict__ pk64, int cold_below) {
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (p >= n) return;
  const int row = sched[p];
  const int64_t b = row_ptr[row], e = row_ptr[row + 1];
  const int64_t o = sptr[p];
  for (int64_t t = b + lane; t < e; t += 64) {
    const int c0 = col_idx[t];
    const int c = (row_ptr[c0 + 1] - row_ptr[c0] < cold_below) ? (int)((unsigned)c0 | 0x80000000u)
                                                               : c0;
    const double w = w64[t];
    if (pk32) pk32[o + (t - b)] = PkEnt32{c, (float)w};
    if (pk64) pk64[o + (t - b)] = PkEnt64{c, 0, w};
  }
}

// Upper-triangle copy: of every stored pair (i, j), (j, i) the one entry whose
// column comes later in the order of the nodes by (degree, id) -- the strict
// upper triangle of A with the nodes in that order.  With A symmetric and no
// self-loop, sum_ij w_ij V_ic V_jd = sum over the copy of w_ij (V_ic V_jd +
// V_jc V_id), so the products with A V of the line searches need only these
// entries, and each row gathers its neighbours of larger degree: the rows that
// are gathered most anyway.  Per row: the number of such entries; flags |= 1
// if any row has a self-loop (the copy is then not built).
// whether column j of row i (degree di) belongs to the copy: j after i by (degree, id)
__device__ inline bool upper_of(const int32_t* __restrict__ row_ptr, int i, int di, int j) {
  const int dj = row_ptr[j + 1] - row_ptr[j];
  return dj > di || (dj == di && j > i);
}

__global__ void graph_upper_count_kernel(int64_t n, const int32_t* __restrict__ row_ptr,
                                         const int32_t* __restrict__ col_idx,
                                         int32_t* __restrict__ ucnt, int* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  bool loop = false;
  const int di = row_ptr[i + 1] - row_ptr[i];
  for (int64_t t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
    const int j = col_idx[t];
    c += upper_of(row_ptr, (int)i, di, j) ? 1 : 0;
    loop = loop || j == i;
  }
  ucnt[i] = c;
  if (loop) atomicOr(flags, 1);
}

// the copy's entries of the row at upper position p (a wavefront per
// position), in their CSR order, compacted to the packed stream at usptr[p];
// cold marks as in graph_pack_kernel
__global__ void graph_pack_upper_kernel(int64_t nu, const int32_t* __restrict__ usched,
                                        const int32_t* __restrict__ row_ptr,
                                        const int32_t* __restrict__ col_idx,
                                        const double* __restrict__ w64,
                                        const int32_t* __restrict__ usptr,
                                        PkEnt32* __restrict__ pk32, PkEnt64* __restrict__ pk64,
                                        int cold_below) {
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x & 63;
  if (p >= nu) return;  // uniform over the wavefront
  const int row = usched[p];
  const int64_t b = row_ptr[row], e = row_ptr[row + 1];
  const int drow = (int)(e - b);
  int64_t o = usptr[p];
  for (int64_t base = b; base < e; base += 64) {
    const int64_t t = base + lane;
    const int c0 = t < e ? col_idx[t] : -1;
    const bool keep = c0 >= 0 && c0 != row && upper_of(row_ptr, row, drow, c0);
    const unsigned long long m = __ballot(keep);
    if (keep) {
      const int64_t at = o + __popcll(m & ((1ull << lane) - 1ull));
      const int c = (row_ptr[c0 + 1] - row_ptr[c0] < cold_below)
                        ? (int)((unsigned)c0 | 0x80000000u)
                        : c0;
      const double w = w64[t];
      if (pk32) pk32[at] = PkEnt32{c, (float)w};
      if (pk64) pk64[at] = PkEnt64{c, 0, w};
    }
    o += __popcll(m);
  }
}

hipError_t launch_graph_upper_count(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                    int32_t* ucnt, int* flags, hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(graph_upper_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, row_ptr,
                     col_idx, ucnt, flags);
  return hipGetLastError();
}

hipError_t launch_graph_pack_upper(int64_t nu, const int32_t* usched, const int32_t* row_ptr,
                                   const int32_t* col_idx, const double* w64,
                                   const int32_t* usptr, void* pk32, void* pk64, int cold_below,
                                   hipStream_t s) {
  const int64_t nb = (nu + 3) / 4;
  hipLaunchKernelGGL(graph_pack_upper_kernel, dim3((unsigned)nb), dim3(256), 0, s, nu, usched,
                     row_ptr, col_idx, w64, usptr, static_cast<PkEnt32*>(pk32),
                     static_cast<PkEnt64*>(pk64), cold_below);
  return hipGetLastError();
}

hipError_t launch_graph_check(int64_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, const double* vals, double* deg,
                              int* flags, hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(graph_check_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, nnz, row_ptr,
                     col_idx, vals, deg, flags);
  return hipGetLastError();
}

hipError_t launch_graph_symcheck(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                 const double* vals, int* flags, hipStream_t s) {
  // the sortedness bit was set by the check kernel; read on the device
  int host_flags = 0;
  hipError_t e = hipMemcpyAsync(&host_flags, flags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int sorted = (host_flags & kGraphUnsorted) ? 0 : 1;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(graph_symcheck_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, row_ptr,
                     col_idx, vals, sorted, flags);
  return hipGetLastError();
}

hipError_t launch_graph_weights(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
                                const double* vals, const double* deg, double* dinv,
                                double* w64, double* normA2_parts, hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(graph_weights_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, row_ptr,
                     col_idx, vals, deg, dinv, w64, normA2_parts);
  return hipGetLastError();
}

hipError_t launch_graph_pack(int64_t n, const int32_t* sched, const int32_t* row_ptr,
                             const int32_t* col_idx, const double* w64, const int32_t* sptr,
                             void* pk32, void* pk64, int cold_below, hipStream_t s) {
  const int64_t nb = (n + 3) / 4;
  hipLaunchKernelGGL(graph_pack_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, sched, row_ptr,
                     col_idx, w64, sptr, static_cast<PkEnt32*>(pk32),
                     static_cast<PkEnt64*>(pk64), cold_below);
  return hipGetLastError();
}

}  // namespace ofm
