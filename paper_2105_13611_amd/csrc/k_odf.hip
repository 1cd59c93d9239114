// ODF reduction (gfx950): floor, per-bin ascending sort, sub-bin means.
//
// Sec. 2.3 of the paper: the fine-grid opacities of a bin are sorted in
// ascending order and split into sub-bins whose widths are fractions of the
// bin; each sub-bin is averaged with the geometric mean (default) or the
// arithmetic mean.  A sorted point i covers [i, i+1) on the sorted axis and
// contributes to sub-bin s with the length of its overlap with
// [F_{s-1} n, F_s n), so fractional sub-bin borders are exact.  Values are
// floored at cutoff * kappa_c(lambda_j) first: below it the line opacity is
// not resolved by the pre-selection (Sec. 4.3); the plan tabulates that
// floor once per fine point (k_floor), in the path's type, and both the ODF
// and the pre-tabulated output read it.
//
// One workgroup per (bin, point).  Keys are the raw bits of the positive
// floored values (FP32 as u32, FP64 as u64), which order like the values;
// they are bitonic-sorted in LDS, padded with all-ones keys to a power of
// two.  Bins too large for LDS sort in a global scratch slab with the same
// network.  Step sums are FP64 in a fixed reduction order.
//
// In LDS, key i sits at i + i / (128 B / key size): one unused key after
// every 128 bytes.  The passes that load 16 consecutive keys per thread
// (the last pass of every stage) would otherwise put the lanes of a
// half-wave on 2 of the 32 banks (u32 keys; 1 of 16 bank pairs for u64);
// with the gap they fall on distinct banks.
#include <algorithm>

#include "odf_internal.h"

namespace odf {

namespace {

constexpr int kOdfThreads = 256;

// Bitonic network over npow2 keys, up to four consecutive steps of a stage
// per pass through memory.  Steps j = 2^h, ..., 2^l of stage k (h - l < 4)
// only ever pair keys of a group {base + c 2^l : c < 2^(h-l+1)}, base with
// bits l .. h clear; all keys of a group share bit k of their index, so
// they sort in one direction (ascending where it is clear).  Each thread
// loads whole groups into registers, runs those steps there (the same
// compare-exchanges, in the same order, as one pass per step) and stores
// them back: one barrier per pass instead of one per step, and a quarter of
// the LDS traffic.
template <bool kPad, typename K>
__device__ __forceinline__ int kidx(int i) {
  return kPad ? i + (i >> (sizeof(K) == 4 ? 5 : 4)) : i;
}

// keys in LDS for a bin of npow2 keys (with the gaps)
template <typename K>
__host__ __device__ inline int lds_keys(int npow2) {
  return npow2 + (npow2 >> (sizeof(K) == 4 ? 5 : 4));
}

template <int M, bool kPad, typename K>
__device__ __forceinline__ void bitonic_pass(K* a, int npow2, int k, int l) {
  constexpr int G = 1 << M;
  const int ng = npow2 >> M;
  const int jl = 1 << l;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    // g with M zero bits inserted at bit l
    const int base = ((g >> l) << (l + M)) | (g & (jl - 1));
    const bool up = (base & k) == 0;
    K r[G];
#pragma unroll
    for (int c = 0; c < G; ++c) r[c] = a[kidx<kPad, K>(base + c * jl)];
#pragma unroll
    for (int t = M - 1; t >= 0; --t) {
#pragma unroll
      for (int c = 0; c < G; ++c) {
        if (c & (1 << t)) continue;
        const K x = r[c], y = r[c + (1 << t)];
        const K lo = x < y ? x : y, hi = x < y ? y : x;
        r[c] = up ? lo : hi;
        r[c + (1 << t)] = up ? hi : lo;
      }
    }
#pragma unroll
    for (int c = 0; c < G; ++c) a[kidx<kPad, K>(base + c * jl)] = r[c];
  }
}

template <bool kPad, typename K>
__device__ void bitonic_sort(K* a, int npow2) {
  int logn = 0;
  while ((1 << logn) < npow2) ++logn;
  for (int kl = 1; kl <= logn; ++kl) {
    const int k = 1 << kl;
    for (int h = kl - 1; h >= 0;) {
      const int m = min(4, h + 1);
      const int l = h - m + 1;
      if (m == 4) bitonic_pass<4, kPad>(a, npow2, k, l);
      else if (m == 3) bitonic_pass<3, kPad>(a, npow2, k, l);
      else if (m == 2) bitonic_pass<2, kPad>(a, npow2, k, l);
      else bitonic_pass<1, kPad>(a, npow2, k, l);
      __syncthreads();
      h = l - 1;
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

// Floor, sort and sub-bin means of bin b at point p, its keys in a (LDS with
// gaps where kPad, else a global slab).
template <bool kPad, typename T, typename K>
__device__ __forceinline__ void odf_bin(const Params& P, const T* __restrict__ kp, T* __restrict__ out,
                                        int b, int p, int64_t e0, int n, int npow2, K* a,
                                        double* red) {
  const T* __restrict__ fl = static_cast<const T*>(P.floor);
  for (int i = threadIdx.x; i < npow2; i += blockDim.x) {
    K key = ~(K)0;
    if (i < n) {
      const int64_t j = e0 + i;
      const T v = kp[j];
      const T f = fl[j];
      key = value_key(v > f ? v : f);
    }
    a[kidx<kPad, K>(i)] = key;
  }
  __syncthreads();
  bitonic_sort<kPad>(a, npow2);
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
        const double v = key_value(a[kidx<kPad, K>(i)]);
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
  const T* kp = kappa + (int64_t)p * kappa_stride;
  if (npow2 <= lds_cap)
    odf_bin<true>(P, kp, out, b, p, e0, n, npow2, reinterpret_cast<K*>(smem), red);
  else   // bins too large for LDS: a private slab of the global scratch
    odf_bin<false>(P, kp, out, b, p, e0, n, npow2,
                   gscratch + (int64_t)p * gscratch_stride + goff[b], red);
}

// The floor cutoff * kappa_c(lambda_j), kappa_c = kc_ref (lambda / kc_lref)^kc_power
// at lambda_j = lambda_1 q^j, rounded once to the path's type.
template <typename T>
__global__ __launch_bounds__(256) void k_floor(Params P, T* __restrict__ out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.N;
       j += (int64_t)gridDim.x * blockDim.x) {
    const double lam = P.lambda_first_nm * exp((double)j * P.lnq);
    out[j] = (T)(P.cutoff * (P.kc_ref * pow(lam / P.kc_lref, P.kc_power)));
  }
}

// Pre-tabulated high-resolution opacity (Sec. 4.1): every fine point is a
// bin of its own with one sub-bin, whose mean is the floored value itself.
// The floor is the table k_odf reads, so the result equals, bit for bit, the
// arithmetic-mean ODF of one-point bins.  Memory-bound: two reads and one
// write per fine point, coalesced, one point of the batch per grid row.
template <typename T>
__global__ __launch_bounds__(256) void k_fine(Params P, const T* __restrict__ kappa,
                                              int64_t kappa_stride, T* __restrict__ out) {
  const int p = blockIdx.y;
  const T* kp = kappa + (int64_t)p * kappa_stride;
  T* op = out + (int64_t)p * P.N;
  const T* __restrict__ fl = static_cast<const T*>(P.floor);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.N;
       j += (int64_t)gridDim.x * blockDim.x) {
    const T v = kp[j];
    const T f = fl[j];
    op[j] = v > f ? v : f;
  }
}

}  // namespace

hipError_t launch_floor(hipStream_t st, const Params& P, void* floor) {
  if (P.N == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((P.N + 255) / 256, 4096);
  if (P.precision == 1)
    hipLaunchKernelGGL(k_floor<float>, dim3((unsigned)blocks), dim3(256), 0, st, P, (float*)floor);
  else
    hipLaunchKernelGGL(k_floor<double>, dim3((unsigned)blocks), dim3(256), 0, st, P, (double*)floor);
  return hipGetLastError();
}

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
    const size_t shmem =
        npow2 <= lds_cap ? (size_t)(P.precision == 1 ? lds_keys<uint32_t>(npow2) : lds_keys<uint64_t>(npow2)) * key_bytes
                         : 0;
    const int max_shmem =
        (P.precision == 1 ? lds_keys<uint32_t>(lds_cap) : lds_keys<uint64_t>(lds_cap)) * key_bytes;
    dim3 grid(cnt, n_points);
    const int32_t* bins = C.bins + C.offset[c];
    if (P.precision == 1) {
      auto k = k_odf<float, uint32_t>;
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         max_shmem);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k, grid, dim3(kOdfThreads), shmem, st, P, (const float*)kappa, kappa_stride,
                         (float*)out, bins, lds_cap, (uint32_t*)gscratch, goff, gscratch_stride);
    } else {
      auto k = k_odf<double, uint64_t>;
      hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         max_shmem);
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
