// Parity-fused pass for small orders: one workgroup applies S^o_tau_o and then
// S^e_tau_e (Sect. 4.3, eqs. solution_operator_odd/_even) to one spatial tile,
// reading every moment once and writing every moment once (2 s bytes per
// update instead of the 3 s of two separate sweeps).
//
// All moments of the tile and a two-point halo are staged in LDS.  The odd
// update is computed on the tile and a one-point ring around it (the even
// update of the tile reads odd values one point outside it); the even update
// then runs on the tile.  On an extrapolation axis a ring position outside
// the grid repeats the nearest grid point, as the separate even sweep's
// staging map does; on a periodic axis the wrapped staging keeps neighbours
// adjacent, so ring values are the true ones.  Every point's arithmetic is
// the separate sweeps' (same coefficients, same order of terms), so the
// results are bitwise equal.  Neighbouring tiles read each other's halos, so
// the pass reads one state buffer and writes the other.
#include "device.hpp"
#include "kernels.hpp"

namespace starmap {

namespace {

constexpr int kThreads = 256;

// Coupling record of one moment, four int4 (host layout in plan_fused):
//   {gx, gy, decay plane, source plane or -1}, {n_x, n_y, 0, 0},
//   x couplings {2 j + o}, y couplings {2 j + o}
// where j is the coupled moment and o = 1 when that moment is cell centred
// along the derivative's axis (its backward neighbour is one point lower).
struct MomentRec {
  int4 g, n, jx, jy;
};

__device__ __forceinline__ MomentRec moment_rec(cptr<int> tab, int k) {
  return MomentRec{rec4(tab, 4 * k), rec4(tab, 4 * k + 1), rec4(tab, 4 * k + 2), rec4(tab, 4 * k + 3)};
}

__device__ __forceinline__ int pick(const int4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(kThreads)
fused_kernel(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ src,
             const typename ComputeOf<T>::type* __restrict__ decay, const int* tab_arg,
             const typename ComputeOf<T>::type* coef_arg, const int* order_arg,
             const FusedScalars<typename ComputeOf<T>::type> a) {
  using C = typename ComputeOf<T>::type;
  constexpr int W2 = TX + 4, H2 = TY + 4, PL = W2 * H2;  // staged tile with a two-point halo
  constexpr int RW = TX + 2, RH = TY + 2, RN = RW * RH;  // tile and one-point ring
  constexpr int RS = (RN + kThreads - 1) / kThreads;     // ring points per thread
  static_assert(TX * TY == kThreads, "one tile point per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  T* L = reinterpret_cast<T*>(smem);
  const cptr<int> tab = (cptr<int>)tab_arg;
  const cptr<int> order = (cptr<int>)order_arg;
  const cptr<C> coef = (cptr<C>)coef_arg;
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % a.ntx) * TX, y0 = (tile / a.ntx) * TY;
  const uint32_t ps = a.ps;

  // 1. stage every moment of the tile and its halo: planes in the outer loop
  //    (uniform grid classes), several planes' loads in flight per thread
  {
    constexpr int E = (PL + kThreads - 1) / kThreads;  // points per thread and plane
    constexpr int B = 4;                                // planes per batch
    for (int j0 = 0; j0 < a.nmom; j0 += B) {
      T v[B][E];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int j = j0 + b;
        if (j < a.nmom) {
          const int4 g = rec4(tab, 4 * j);
          const T* up = plane_at(uin, j, ps);
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const int e = tid + q * kThreads;
            if (e < PL) {
              const int lx = e % W2 - 2, ly = e / W2 - 2;
              const int X = map_axis(x0 + lx, a.nx, a.px, g.x == 1), Y = map_axis(y0 + ly, a.ny, a.py, g.y == 1);
              v[b][q] = up[uint32_t(Y * a.pitch + X)];
            }
          }
        }
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int j = j0 + b;
        if (j < a.nmom) {
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const int e = tid + q * kThreads;
            if (e < PL) L[j * PL + e] = v[b][q];
          }
        }
      }
    }
  }
  __syncthreads();

  // The flux sum of moment k (record r) at staged position p = (ly + 2) W2 +
  // lx + 2 from the staged planes of the other parity, terms in row order.
  auto flux = [&](const MomentRec& r, cptr<C> cf, int p) {
    C W = C(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // D_x couplings
      if (i < r.n.x) {
        const int e = pick(r.jx, i), q = (e >> 1) * PL + p - (e & 1);
        W = couple(W, cf[i], to_c(L[q + 1]), to_c(L[q]));
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // D_y couplings
      if (i < r.n.y) {
        const int e = pick(r.jy, i), q = (e >> 1) * PL + p - (e & 1) * W2;
        W = couple(W, cf[4 + i], to_c(L[q + W2]), to_c(L[q]));
      }
    }
    return W;
  };

  // 2. odd moments on the tile and its ring; decay factors cached per output
  //    grid of the parity (slot: cell centred along x or not)
  {
    C cc[RS][2], ce[RS][2];
    int cdk[2] = {-1, -1};
    for (int q = 0; q < a.nodd; ++q) {
      const int k = order[q];
      const MomentRec r = moment_rec(tab, k);
      const cptr<C> cf = cat(coef, uint32_t(k) * uint32_t(8 * sizeof(C)));
      const int g = r.g.x == 1 ? 0 : 1;
      const bool fresh = r.g.z != cdk[g];
      cdk[g] = r.g.z;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int e = tid + s * kThreads;
        if (e < RN) {
          const int lx = e % RW - 1, ly = e / RW - 1;
          const int X = map_axis(x0 + lx, a.nx, a.px, r.g.x == 1), Y = map_axis(y0 + ly, a.ny, a.py, r.g.y == 1);
          const uint32_t off = uint32_t(Y * a.pitch + X);
          const int p = (ly + 2) * W2 + lx + 2;
          C W = flux(r, cf, p);
          if (r.g.w >= 0) W += to_c(plane_at(src, r.g.w, ps)[off]);
          if (fresh) {
            cc[s][g] = plane_at(decay, r.g.z, ps)[off];
            ce[s][g] = expm1div(-cc[s][g] * a.tau_odd);
          }
          T* u = L + k * PL + p;
          *u = from_c<T>(sub_step(to_c(*u), W, cc[s][g], ce[s][g], a.tau_odd));
        }
      }
    }
  }
  __syncthreads();
  // 3. ring positions outside the grid on an extrapolation axis take the
  //    value of the grid point they repeat
  if (!a.px || !a.py) {
    for (int q = 0; q < a.nodd; ++q) {
      const int4 g = rec4(tab, 4 * order[q]);
      const int k = order[q];
      for (int e = tid; e < RN; e += kThreads) {
        const int lx = e % RW - 1, ly = e / RW - 1;
        const int mx = a.px ? lx : map_axis(x0 + lx, a.nx, 0, g.x == 1) - x0;
        const int my = a.py ? ly : map_axis(y0 + ly, a.ny, 0, g.y == 1) - y0;
        if (mx != lx || my != ly) L[k * PL + (ly + 2) * W2 + lx + 2] = L[k * PL + (my + 2) * W2 + mx + 2];
      }
    }
    __syncthreads();
  }

  // 4. even moments on the tile (one point per thread)
  const int tx = tid % TX, ty = tid / TX;
  {
    C cc[2], ce[2];
    int cdk[2] = {-1, -1};
    const int p = (ty + 2) * W2 + tx + 2;
    for (int q = a.nodd; q < a.nmom; ++q) {
      const int k = order[q];
      const MomentRec r = moment_rec(tab, k);
      const cptr<C> cf = cat(coef, uint32_t(k) * uint32_t(8 * sizeof(C)));
      const int g = r.g.x == 1 ? 0 : 1;
      const int X = map_axis(x0 + tx, a.nx, a.px, r.g.x == 1), Y = map_axis(y0 + ty, a.ny, a.py, r.g.y == 1);
      const uint32_t off = uint32_t(Y * a.pitch + X);
      C W = flux(r, cf, p);
      if (r.g.w >= 0) W += to_c(plane_at(src, r.g.w, ps)[off]);
      if (r.g.z != cdk[g]) {
        cc[g] = plane_at(decay, r.g.z, ps)[off];
        ce[g] = expm1div(-cc[g] * a.tau_even);
        cdk[g] = r.g.z;
      }
      T* u = L + k * PL + p;
      *u = from_c<T>(sub_step(to_c(*u), W, cc[g], ce[g], a.tau_even));
    }
  }
  __syncthreads();

  // 5. every moment's tile points that exist on its grid
  for (int k = 0; k < a.nmom; ++k) {
    const int4 g = rec4(tab, 4 * k);
    const int nxk = g.x == 1 ? a.nx : a.nx + 1 - a.px, nyk = g.y == 1 ? a.ny : a.ny + 1 - a.py;
    const int X = x0 + tx, Y = y0 + ty;
    if (X < nxk && Y < nyk) plane_at(uout, k, ps)[uint32_t(Y * a.pitch + X)] = L[k * PL + (ty + 2) * W2 + tx + 2];
  }
}

template <typename T>
size_t lds_t(int nmom) {
  return size_t(nmom) * (32 + 4) * (8 + 4) * sizeof(T);
}

template <typename T>
hipError_t launch_t(const FusedArgs& f, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  const size_t lds = lds_t<T>(f.nmom);
  static size_t attr = 0;
  if (lds > attr) {
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (lds > size_t(max_lds)) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_kernel<T, 32, 8>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
    if (e != hipSuccess) return e;
    attr = size_t(max_lds);
  }
  FusedScalars<C> sc;
  sc.ps = f.ps;
  sc.pitch = f.pitch;
  sc.nx = f.nx;
  sc.ny = f.ny;
  sc.px = f.px;
  sc.py = f.py;
  sc.ntx = f.ntx;
  sc.nty = f.nty;
  sc.nmom = f.nmom;
  sc.nodd = f.nodd;
  sc.tau_odd = C(f.tau_odd);
  sc.tau_even = C(f.tau_even);
  hipLaunchKernelGGL((fused_kernel<T, 32, 8>), dim3(f.ntx * f.nty), dim3(kThreads), lds, stream,
                     static_cast<const T*>(f.uin), static_cast<T*>(f.uout), static_cast<const T*>(f.src),
                     static_cast<const C*>(f.decay), f.tab, static_cast<const C*>(f.coef), f.order, sc);
  return hipGetLastError();
}

}  // namespace

size_t fused_lds_bytes(int storage, int nmom) {
  switch (storage) {
    case STORE_FP64: return lds_t<double>(nmom);
    case STORE_FP32: return lds_t<float>(nmom);
    case STORE_BF16: return lds_t<bf16>(nmom);
  }
  return 0;
}

hipError_t launch_fused(int storage, const FusedArgs& f, hipStream_t stream) {
  if (f.nmom < 1 || f.nodd < 0 || f.nodd > f.nmom || f.ntx < 1 || f.nty < 1) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return launch_t<double>(f, stream);
    case STORE_FP32: return launch_t<float>(f, stream);
    case STORE_BF16: return launch_t<bf16>(f, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace starmap
