// Float map-reduce of Section 4.2: the sum over i = 1..n of a term mapped from its index,
// either sqrt(i) or (-1)^(i+1) / i (the alternating harmonic series, whose limit is ln 2),
// in binary64. There is no input in memory: the work is the terms' arithmetic, so the kernel
// is bound by fp64 vector issue (square root and division expand to several instructions).
//
// Layout: T = 256 * G threads (G = min(kFoldMaxBlocks, ceil(n / 256)) workgroups); thread t
// adds the consecutive terms [1 + t*m, 1 + (t+1)*m) of its share (m = ceil(n / T)) in index
// order. A wave adds its 64 partials in a fixed butterfly, a workgroup its 4 wave sums, and
// a second one-workgroup kernel adds the G workgroup sums in a fixed tree. The result is the
// same on every run (no atomics); it differs from the exactly rounded sum of the rounded terms
// by at most (m + 23) u sum|term| (u = 2^-53), the depth of that addition tree.
#include "../../include/wc_fold.h"
#include "wc_internal.h"

namespace wc {

void set_last_hip(int32_t e);  // wc_api.hip

namespace {

constexpr uint64_t kFoldMaxBlocks = 2048;

// term i; x == (double)i exactly (indices stay below 2^53)
WC_DEV double fold_term(uint32_t kind, uint64_t i, double x) {
  if (kind == 0) return __builtin_sqrt(x);  // correctly rounded
  const double r = 1.0 / x;                 // correctly rounded (IEEE division)
  return (i & 1) ? r : -r;
}

WC_DEV double wave_sum(double v) {
  // fixed butterfly over the 64 lanes: every lane ends with the same total
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <uint32_t KIND>
__global__ __launch_bounds__(256) void fold_partial_kernel(uint64_t n, uint64_t m, double* part) {
  __shared__ double s_w[4];
  const uint64_t t = blockIdx.x * 256ull + threadIdx.x;
  const uint64_t a = 1 + t * m;
  const uint64_t b = min(n + 1, a + m);  // a > n: no terms
  double s = 0.0, x = (double)a;
  for (uint64_t i = a; i < b; ++i, x += 1.0) s += fold_term(KIND, i, x);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

__global__ __launch_bounds__(256) void fold_final_kernel(const double* part, uint32_t g,
                                                         double* out) {
  __shared__ double s_w[4];
  // thread j adds partials j, j + 256, ... in order, then the fixed tree
  double s = 0.0;
  for (uint32_t k = threadIdx.x; k < g; k += 256) s += part[k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

}  // namespace

void fold_layout(uint64_t n, uint32_t* blocks, uint64_t* per_thread) {
  uint64_t g = (n + 255) / 256;
  if (g > kFoldMaxBlocks) g = kFoldMaxBlocks;
  if (g == 0) g = 1;
  const uint64_t threads = g * 256;
  *blocks = (uint32_t)g;
  *per_thread = (n + threads - 1) / threads;
}

hipError_t launch_fold(uint32_t kind, uint64_t n, double* d_out, double* d_part, hipStream_t s) {
  uint32_t g;
  uint64_t m;
  fold_layout(n, &g, &m);
  if (kind == 0)
    hipLaunchKernelGGL(fold_partial_kernel<0>, dim3(g), dim3(256), 0, s, n, m, d_part);
  else
    hipLaunchKernelGGL(fold_partial_kernel<1>, dim3(g), dim3(256), 0, s, n, m, d_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fold_final_kernel, dim3(1), dim3(256), 0, s, d_part, g, d_out);
  return hipGetLastError();
}

}  // namespace wc

extern "C" {

wc_status wc_fold_sum_plan(uint64_t n, uint64_t* workspace_bytes) {
  if (!workspace_bytes) return WC_EINVAL;
  uint32_t g;
  uint64_t m;
  wc::fold_layout(n, &g, &m);
  *workspace_bytes = (uint64_t)g * sizeof(double);
  return WC_OK;
}

wc_status wc_fold_sum(uint32_t kind, uint64_t n, double* d_out, void* d_workspace,
                      uint64_t workspace_bytes, void* stream) {
  if (kind > WC_FOLD_ALT_HARMONIC || n > (1ull << 53) || !d_out || !d_workspace ||
      ((uintptr_t)d_workspace & 7))
    return WC_EINVAL;
  uint64_t need = 0;
  wc_fold_sum_plan(n, &need);
  if (workspace_bytes < need) return WC_EINVAL;
  hipError_t e = wc::launch_fold(kind, n, d_out, (double*)d_workspace, (hipStream_t)stream);
  if (e != hipSuccess) {
    wc::set_last_hip((int32_t)e);
    return WC_EDEVICE;
  }
  return WC_OK;
}

}  // extern "C"
