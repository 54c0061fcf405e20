// Decay and source planes of time-separable data, formed on the device once
// per step (time-dependent data are frozen at t + dt/2 for a step, Sect. 5.7):
// each output plane is a short linear combination of basis planes g_i whose
// time factors a_i(t + dt/2) arrive as kernel arguments.  HBM-bound: per
// output point one read per entry and one write.
#include "device.hpp"
#include "kernels.hpp"

namespace starmap {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;

// blockIdx.y: one (output, destination plane) pair of the list; blockIdx.x:
// kThreads * kPerThread consecutive points of the plane.  The entry range is
// uniform over the block.
template <typename C, typename To>
__global__ void __launch_bounds__(kThreads) combine_kernel(CombineArgs a) {
  const int o = a.list[2 * blockIdx.y], dst = a.list[2 * blockIdx.y + 1];
  const int e0 = a.first[o], e1 = a.first[o + 1];
  const C* basis = static_cast<const C*>(a.basis);
  To* out = static_cast<To*>(a.out) + int64_t(dst) * a.plane_stride;
  const int64_t base = int64_t(blockIdx.x) * (kThreads * kPerThread) + threadIdx.x;
  C acc[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) acc[r] = C(a.cst[o]);
  for (int e = e0; e < e1; ++e) {
    const int b = a.entries[3 * e], term = a.entries[3 * e + 1], sign = a.entries[3 * e + 2];
    const C coef = C(double(sign) * (term >= 0 ? a.a[term] : 1.0));
    const C* g = basis + int64_t(b) * a.plane_stride;
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
      const int64_t i = base + r * kThreads;
      if (i < a.plane_stride) acc[r] = fma(coef, g[i], acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const int64_t i = base + r * kThreads;
    if (i < a.plane_stride) out[i] = from_c<To>(acc[r]);
  }
}

template <typename C, typename To>
hipError_t launch_t(const CombineArgs& a, hipStream_t stream) {
  const int64_t per_block = kThreads * kPerThread;
  const dim3 grid(unsigned((a.plane_stride + per_block - 1) / per_block), unsigned(a.nlist));
  hipLaunchKernelGGL((combine_kernel<C, To>), grid, dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_combine(int storage, bool to_compute_type, const CombineArgs& a, hipStream_t stream) {
  if (a.nlist < 1 || a.nlist > 65535 || a.plane_stride < 1) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return launch_t<double, double>(a, stream);
    case STORE_FP32: return launch_t<float, float>(a, stream);
    case STORE_BF16:
      return to_compute_type ? launch_t<float, float>(a, stream) : launch_t<float, bf16>(a, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace starmap
