// ODF reduction (gfx950): floor, per-bin ascending sort, sub-bin means.
//
// Sec. 2.3 of the paper: the fine-grid opacities of a bin are sorted in
// ascending order and split into sub-bins whose widths are fractions of the
// bin; each sub-bin is averaged with the geometric mean (default) or the
// arithmetic mean.  A sorted point i covers [i, i+1) on the sorted axis and
// contributes to sub-bin s with the length of its overlap with
// [F_{s-1} n, F_s n), so fractional sub-bin borders are exact.  Values are
// floored at cutoff * kappa_c(lambda_j) first: below it the line opacity is
// not resolved by the pre-selection (Sec. 4.3).
//
// One workgroup per (bin, point).  Keys are the raw bits of the positive
// floored values (FP32 as u32, FP64 as u64), which order like the values;
// they are bitonic-sorted in LDS, padded with all-ones keys to a power of
// two.  Bins too large for LDS sort in a global scratch slab with the same
// network.  Step sums are FP64 in a fixed reduction order.
#include <algorithm>

#include "odf_internal.h"

namespace odf {

namespace {

constexpr int kOdfThreads = 256;

// Bitonic network over npow2 keys.  Each step of stage (k, j) is npow2/2
// independent compare-exchanges of the pairs (i, i + j) with bit j of i
// clear; a thread takes pairs by pair index, so no thread idles, and writes
// min and max back without a branch (ascending where bit k of i is clear).
template <typename K>
__device__ void bitonic_sort(K* a, int npow2) {
  const int half = npow2 >> 1;
  for (int k = 2; k <= npow2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < half; q += blockDim.x) {
        const int i = q + (q & ~(j - 1));   // insert a zero at bit j
        const K ai = a[i], aj = a[i + j];
        const K lo = ai < aj ? ai : aj, hi = ai < aj ? aj : ai;
        const bool up = (i & k) == 0;
        a[i] = up ? lo : hi;
        a[i + j] = up ? hi : lo;
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ double key_value(uint32_t k) { return (double)__uint_as_float(k); }
__device__ __forceinline__ double key_value(uint64_t k) { return __longlong_as_double((long long)k); }
__device__ __forceinline__ uint32_t value_key(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint64_t value_key(double v) { return (uint64_t)__double_as_longlong(v); }

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    red[0] = t;
  }
  __syncthreads();
  t = red[0];
  __syncthreads();
  return t;
}

template <typename T, typename K>
__global__ __launch_bounds__(kOdfThreads) void k_odf(Params P, const T* __restrict__ kappa,
                                                     int64_t kappa_stride, T* __restrict__ out,
                                                     const int32_t* __restrict__ bins,
                                                     int lds_cap, K* __restrict__ gscratch,
                                                     const int64_t* __restrict__ goff,
                                                     int64_t gscratch_stride) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kOdfThreads / 64];
  const int b = bins[blockIdx.x], p = blockIdx.y;
  const int64_t e0 = P.edges[b], e1 = P.edges[b + 1];
  const int n = (int)(e1 - e0);
  int npow2 = 1;
  while (npow2 < n) npow2 <<= 1;
  K* a;
  if (npow2 <= lds_cap) {
    a = reinterpret_cast<K*>(smem);
  } else {
    // bins too large for LDS: a private slab of the global scratch
    a = gscratch + (int64_t)p * gscratch_stride + goff[b];
  }
  const T* kp = kappa + (int64_t)p * kappa_stride;
  for (int i = threadIdx.x; i < npow2; i += blockDim.x) {
    K key = ~(K)0;
    if (i < n) {
      const int64_t j = e0 + i;
      const double lam = P.lambda_first_nm * exp((double)j * P.lnq);
      const double fl = P.cutoff * (P.kc_ref * pow(lam / P.kc_lref, P.kc_power));
      const T v = kp[j];
      const T f = (T)fl;
      key = value_key(v > f ? v : f);
    }
    a[i] = key;
  }
  __syncthreads();
  bitonic_sort(a, npow2);
  const int S = P.n_steps;
  const double dn = (double)n;
  for (int s = 0; s < S; ++s) {
    const double lo = P.Fcum[s] * dn, hi = P.Fcum[s + 1] * dn;
    const int i0 = (int)floor(lo);
    const int i1 = min(n, (int)ceil(hi));
    double acc = 0.0;
    for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
      const double w = fmin((double)(i + 1), hi) - fmax((double)i, lo);
      if (w > 0.0) {
        const double v = key_value(a[i]);
        acc += w * (P.mean == 0 ? log(v) : v);
      }
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) {
      const double m = tot / (hi - lo);
      out[((int64_t)p * P.n_bins + b) * S + s] = (T)(P.mean == 0 ? exp(m) : m);
    }
  }
}

// Pre-tabulated high-resolution opacity (Sec. 4.1): every fine point is a
// bin of its own with one sub-bin, whose mean is the floored value itself.
// The floor is taken exactly as in k_odf, so the result equals, bit for bit,
// the arithmetic-mean ODF of one-point bins.  Memory-bound: one read and one
// write per fine point, coalesced, one point of the batch per grid row.
template <typename T>
__global__ __launch_bounds__(256) void k_fine(Params P, const T* __restrict__ kappa,
                                              int64_t kappa_stride, T* __restrict__ out) {
  const int p = blockIdx.y;
  const T* kp = kappa + (int64_t)p * kappa_stride;
  T* op = out + (int64_t)p * P.N;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.N;
       j += (int64_t)gridDim.x * blockDim.x) {
    const double lam = P.lambda_first_nm * exp((double)j * P.lnq);
    const double fl = P.cutoff * (P.kc_ref * pow(lam / P.kc_lref, P.kc_power));
    const T v = kp[j];
    const T f = (T)fl;
    op[j] = v > f ? v : f;
  }
}

}  // namespace

hipError_t launch_fine(hipStream_t st, const Params& P, const void* kappa, int64_t kappa_stride,
                       int32_t n_points, void* out) {
  if (n_points == 0 || P.N == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((P.N + 255) / 256, 2048);
  dim3 grid((unsigned)blocks, n_points);
  if (P.precision == 1)
    hipLaunchKernelGGL(k_fine<float>, grid, dim3(256), 0, st, P, (const float*)kappa, kappa_stride,
                       (float*)out);
  else
    hipLaunchKernelGGL(k_fine<double>, grid, dim3(256), 0, st, P, (const double*)kappa,
                       kappa_stride, (double*)out);
  return hipGetLastError();
}

hipError_t launch_odf(hipStream_t st, const Params& P, const void* kappa, int64_t kappa_stride,
                      int32_t n_points, void* out, const OdfClasses& C, void* gscratch,
                      const int64_t* goff, int64_t gscratch_stride) {
  if (n_points == 0 || P.n_bins == 0) return hipSuccess;
  const int key_bytes = P.precision == 1 ? 4 : 8;
  const int lds_cap = odf_lds_cap(P.precision);
  // one launch per bin-size class, each with the LDS its largest bin needs
  for (int c = 0; c < C.n_classes; ++c) {
    const int cnt = C.count[c];
    if (cnt == 0) continue;
    const int npow2 = C.npow2[c];
    const size_t shmem = npow2 <= lds_cap ? (size_t)npow2 * key_bytes : 0;
    dim3 grid(cnt, n_points);
    const int32_t* bins = C.bins + C.offset[c];
    if (P.precision == 1) {
      auto k = k_odf<float, uint32_t>;
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(lds_cap * key_bytes));
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(kOdfThreads), shmem, st, P, (const float*)kappa, kappa_stride,
                         (float*)out, bins, lds_cap, (uint32_t*)gscratch, goff, gscratch_stride);
    } else {
      auto k = k_odf<double, uint64_t>;
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)(lds_cap * key_bytes));
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(kOdfThreads), shmem, st, P, (const double*)kappa,
                         kappa_stride, (double*)out, bins, lds_cap, (uint64_t*)gscratch, goff,
                         gscratch_stride);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace odf
