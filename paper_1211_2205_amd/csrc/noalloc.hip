// Diagnostics without any device allocation: the FP64 block partials and the
// four results of the diagnostics reduction live in a file-scope device array
// instead of the solver's workspace, for callers that cannot allocate (code
// under stream capture, tight loops, harnesses that forbid allocation).
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Host code never uses the array's name as an address: its
// device address is looked up once per device (with that device current) and
// kept per device.  Every call on one device shares that device's array and
// leaves the last call's contents there; nothing in it needs clearing (every
// partial a call reads was written by the same call).  Calls that overlap on
// one device (two streams, two threads) race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <mutex>

#include "solver.hpp"

namespace starmap {
namespace {

// 65536 blocks of 4 partials, then the 4 results (2 MiB + 32 bytes)
constexpr int kScratchBlocks = 65536;
constexpr size_t kScratchDoubles = size_t(kScratchBlocks) * 4 + 4;

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's array (looked up on first use).
hipError_t scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace starmap

using namespace starmap;
using namespace starmap::detail;

extern "C" int starmap_diagnostics_noalloc(const starmap_solver* cs, double* mass, double* l2, double* maxabs,
                                           int32_t* nonfinite) {
  starmap_solver* s = const_cast<starmap_solver*>(cs);
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (!s->device_ready)
    return fail(STARMAP_ESTATE, "starmap_diagnostics_noalloc: the solver has no device state yet (it would allocate)");
  const int blocks_per_plane = (s->ny + 1 + s->diag_rows_per_block - 1) / s->diag_rows_per_block;
  const int64_t nb = int64_t(s->nmom) * blocks_per_plane;
  if (nb > kScratchBlocks)
    return fail(STARMAP_EINVAL, "starmap_diagnostics_noalloc: " + std::to_string(nb) +
                                    " reduction blocks exceed the static scratch of " +
                                    std::to_string(kScratchBlocks) + " (moments x ceil((ny + 1) / 64))");
  double* scr = nullptr;
  HIP_TRY(scratch_ptr(&scr));
  DiagArgs a;
  a.u = dptr(s, s->off_state);
  // the per-plane extents sit in the workspace, written when the device state was set up
  const size_t geo = s->off_diag + align256(size_t(s->diag_nblocks) * 4 * 8) + 256;
  a.plane_nx = reinterpret_cast<const int*>(dptr(s, geo));
  a.plane_ny = reinterpret_cast<const int*>(dptr(s, geo)) + s->nmom;
  a.nplanes = s->nmom;
  a.plane_stride = s->plane_stride;
  a.pitch = s->pitch;
  a.rows_per_block = s->diag_rows_per_block;
  a.blocks_per_plane = blocks_per_plane;
  a.part = scr;
  a.out = scr + size_t(kScratchBlocks) * 4;
  HIP_TRY(launch_diagnostics(s->storage, a, s->stream));
  double res[4];
  HIP_TRY(hipMemcpyAsync(res, a.out, sizeof(res), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const double area = s->dx * s->dy;
  if (mass) *mass = area * res[0];
  if (l2) *l2 = std::sqrt(area * res[1]);
  if (maxabs) *maxabs = res[2];
  if (nonfinite) *nonfinite = int32_t(res[3]);
  if (res[3] != 0.0) return fail(STARMAP_EUNSTABLE, "non-finite values in the state");
  return STARMAP_OK;
}
