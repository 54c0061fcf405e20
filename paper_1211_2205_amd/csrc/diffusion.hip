// Diffusion step of the diffusion-corrected P_N model (D_N), one of the
// moment models the paper names as fitting its splitting (Sect. 7): on every
// moment of the highest order N,
//   u <- u + tau kappa (D_xx u + D_yy u),
// three-point second differences on the moment's own grid, explicit in time.
// Boundaries use the sweep's staging index map (wrap for periodic axes,
// repeat the boundary point for extrapolation axes).  The update reads
// neighbours, so it writes scratch planes that a second kernel copies back.
// HBM-bound: per point one read of u (neighbours come from cache), one of
// kappa, one scratch write, then one scratch read and one state write.
#include "device.hpp"
#include "kernels.hpp"

namespace starmap {

namespace {

constexpr int kThreads = 256;

struct PlaneGeo {
  int k, cell_x, cell_y, nxk, nyk;
};

__device__ __forceinline__ PlaneGeo plane_geo(const DiffusionArgs& a, int j) {
  PlaneGeo g;
  g.k = a.tab[3 * j];
  g.cell_x = a.tab[3 * j + 1] == 1;
  g.cell_y = a.tab[3 * j + 2] == 1;
  g.nxk = g.cell_x ? a.nx : a.nx + 1 - a.px;
  g.nyk = g.cell_y ? a.ny : a.ny + 1 - a.py;
  return g;
}

// blockIdx.y: plane j; the points of its grid in grid-stride order
template <typename T>
__global__ void __launch_bounds__(kThreads) diffusion_kernel(DiffusionArgs a) {
  using C = typename ComputeOf<T>::type;
  const int j = blockIdx.y;
  const PlaneGeo g = plane_geo(a, j);
  const T* u = static_cast<const T*>(a.u) + int64_t(g.k) * a.plane_stride;
  const C* kap = static_cast<const C*>(a.kappa) + int64_t(j) * a.plane_stride;
  T* out = static_cast<T*>(a.tmp) + int64_t(j) * a.plane_stride;
  const C rdx2 = C(a.rdx2), rdy2 = C(a.rdy2), tau = C(a.tau);
  const int npts = g.nxk * g.nyk;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < npts; i += gridDim.x * kThreads) {
    const int y = i / g.nxk, x = i - y * g.nxk;
    const int xe = map_axis(x + 1, a.nx, a.px, g.cell_x), xw = map_axis(x - 1, a.nx, a.px, g.cell_x);
    const int yn = map_axis(y + 1, a.ny, a.py, g.cell_y), ys = map_axis(y - 1, a.ny, a.py, g.cell_y);
    const int row = y * a.pitch;
    const C c = to_c(u[row + x]);
    const C lx = to_c(u[row + xe]) - C(2) * c + to_c(u[row + xw]);
    const C ly = to_c(u[yn * a.pitch + x]) - C(2) * c + to_c(u[ys * a.pitch + x]);
    out[row + x] = from_c<T>(c + tau * kap[row + x] * (lx * rdx2 + ly * rdy2));
  }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) diffusion_copy_kernel(DiffusionArgs a) {
  const int j = blockIdx.y;
  const PlaneGeo g = plane_geo(a, j);
  T* u = static_cast<T*>(a.u) + int64_t(g.k) * a.plane_stride;
  const T* src = static_cast<const T*>(a.tmp) + int64_t(j) * a.plane_stride;
  const int npts = g.nxk * g.nyk;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < npts; i += gridDim.x * kThreads) {
    const int y = i / g.nxk, x = i - y * g.nxk;
    u[y * a.pitch + x] = src[y * a.pitch + x];
  }
}

template <typename T>
hipError_t launch_t(const DiffusionArgs& a, int max_points, hipStream_t stream) {
  const dim3 grid(unsigned((max_points + kThreads - 1) / kThreads), unsigned(a.nplanes));
  hipLaunchKernelGGL(diffusion_kernel<T>, grid, dim3(kThreads), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diffusion_copy_kernel<T>, grid, dim3(kThreads), 0, stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_diffusion(int storage, const DiffusionArgs& a, int max_points, hipStream_t stream) {
  if (a.nplanes < 1 || a.nplanes > 65535 || max_points < 1) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return launch_t<double>(a, max_points, stream);
    case STORE_FP32: return launch_t<float>(a, max_points, stream);
    case STORE_BF16: return launch_t<bf16>(a, max_points, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace starmap
