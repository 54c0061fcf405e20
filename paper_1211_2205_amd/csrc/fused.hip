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
// the separate sweeps' (same coefficients, same order of terms; padded
// coupling terms have coefficient zero), so for finite states the results are
// bitwise equal.  Neighbouring tiles read each other's halos, so
// the pass reads one state buffer and writes the other.
#include "device.hpp"
#include "kernels.hpp"

namespace starmap {

namespace {

constexpr int kThreads = 256;

// Record of one moment, four int4, in processing order (odd parity first):
//   {gx, gy, decay plane, source plane or -1}, {k, reload, k P, 0},
//   x couplings {j P - o}, y couplings {j P - o R}
// where k is the moment, P the staged plane and R the staged row
// (kFusedPlane, kFusedRow), reload = 1 when the decay plane differs from the
// one last used on its grid within its parity, j a coupled moment and o = 1
// when moment j is cell centred along the derivative's axis (its backward
// neighbour is one point lower): a coupling's LDS pair is (q + 1, q) along x
// and (q + R, q) along y with q = offset + position.  Coupling lists are
// padded to four entries with zero coefficients (a zero term leaves the
// finite sum unchanged).
// Records sit at fixed offsets, so no table read waits on another.  After the
// nmom moment records come nd int4 {gx, gy, 0, 0}: the grid of each decay
// plane.
struct MomentRec {
  int4 g, n, jx, jy;
};

__device__ __forceinline__ MomentRec moment_rec(cptr<int> tab, int q) {
  return MomentRec{rec4(tab, 4 * q), rec4(tab, 4 * q + 1), rec4(tab, 4 * q + 2), rec4(tab, 4 * q + 3)};
}

__device__ __forceinline__ int pick(const int4& v, int i) { return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w; }

// Grid offsets of one position for the four grid classes (cell centred along
// x: bit 0, along y: bit 1).
struct ClassOffsets {
  uint32_t o00, o10, o01, o11;  // o<x class><y class>
  __device__ __forceinline__ uint32_t of(int gx, int gy) const {
    const uint32_t ny = gx == 1 ? o10 : o00, cy = gx == 1 ? o11 : o01;
    return gy == 1 ? cy : ny;
  }
};

// Decay factors of the two grids of one parity at one position (slot 0: cell
// centred along x), held in named registers: selects, no indexed arrays.
template <typename C>
struct DecayCache {
  C c0, e0, c1, e1;
  __device__ __forceinline__ void set(bool slot0, C c, C e) {
    if (slot0) {
      c0 = c;
      e0 = e;
    } else {
      c1 = c;
      e1 = e;
    }
  }
  __device__ __forceinline__ C c(bool slot0) const { return slot0 ? c0 : c1; }
  __device__ __forceinline__ C e(bool slot0) const { return slot0 ? e0 : e1; }
};

template <typename C>
__device__ __forceinline__ ClassOffsets class_offsets(int X, int Y, const FusedScalars<C>& a) {
  const int x0 = map_axis(X, a.nx, a.px, 0), x1 = map_axis(X, a.nx, a.px, 1);
  const int y0 = map_axis(Y, a.ny, a.py, 0), y1 = map_axis(Y, a.ny, a.py, 1);
  return ClassOffsets{uint32_t(y0 * a.pitch + x0), uint32_t(y0 * a.pitch + x1), uint32_t(y1 * a.pitch + x0),
                      uint32_t(y1 * a.pitch + x1)};
}

// B >= nmom: every state plane is staged in one batch of loads.
template <typename T, int TX, int TY, int B>
__global__ void __launch_bounds__(kThreads)
fused_kernel(const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ src,
             const typename ComputeOf<T>::type* __restrict__ decay, const int* tab_arg,
             const typename ComputeOf<T>::type* coef_arg,
             const FusedScalars<typename ComputeOf<T>::type> a) {
  using C = typename ComputeOf<T>::type;
  constexpr int W2 = TX + 4, H2 = TY + 4, PL = W2 * H2;  // staged tile with a two-point halo
  constexpr int RW = TX + 2, RH = TY + 2, RN = RW * RH;  // tile and one-point ring
  constexpr int E = (PL + kThreads - 1) / kThreads;      // staged points per thread and plane
  constexpr int BD = 8;                                  // decay planes staged per batch
  constexpr int G = 4;                                   // moments updated together
  static_assert(TX * TY == kThreads, "one tile point per thread");
  static_assert(PL == kFusedPlane && W2 == kFusedRow, "the host's coupling offsets use the same staged plane");
  static_assert(RN <= 2 * kThreads, "tile and ring within two points per thread");
  extern __shared__ __align__(16) unsigned char smem[];
  using S = typename StagedOf<T>::type;                                // BF16 staged as FP32
  S* L = reinterpret_cast<S*>(smem);                                   // nmom planes of PL
  C* D = reinterpret_cast<C*>(smem + size_t(a.nmom) * PL * sizeof(S));  // nd decay planes of PL
  const cptr<int> tab = (cptr<int>)tab_arg;
  const cptr<C> coef = (cptr<C>)coef_arg;
  const int tid = threadIdx.x;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % a.ntx) * TX, y0 = (tile / a.ntx) * TY;
  const uint32_t ps = a.ps;

  // 1. stage every moment of the tile and its halo, B planes' loads in flight
  {
    ClassOffsets so[E];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const int e = min(tid + q * kThreads, PL - 1);
      so[q] = class_offsets(x0 + e % W2 - 2, y0 + e / W2 - 2, a);
    }
    // All state planes and the first BD decay planes in one batch, further
    // decay planes BD at a time.  Indices past the end repeat the last plane
    // (loads without branches: a load under a branch makes the compiler wait
    // for every earlier load before it); repeated stores write equal values.
    for (int d0 = 0; d0 == 0 || d0 < a.nd; d0 += BD) {
      T v[B][E];
      C w[BD][E];
      if (d0 == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int j = min(b, a.nmom - 1);
          const int4 g = rec4(tab, 4 * j);
          const T* up = plane_at(uin, rec4(tab, 4 * j + 1).x, ps);
#pragma unroll
          for (int q = 0; q < E; ++q) v[b][q] = up[so[q].of(g.x, g.y)];
        }
      }
#pragma unroll
      for (int b = 0; b < BD; ++b) {
        const int d = min(d0 + b, a.nd - 1);
        const int4 g = rec4(tab, 4 * a.nmom + d);
        const C* dp = plane_at(decay, d, ps);
#pragma unroll
        for (int q = 0; q < E; ++q) w[b][q] = dp[so[q].of(g.x, g.y)];
      }
      if (d0 == 0) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int k = rec4(tab, 4 * min(b, a.nmom - 1) + 1).x;
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const int e = tid + q * kThreads;
            if (e < PL) L[k * PL + e] = S(to_c(v[b][q]));
          }
        }
      }
#pragma unroll
      for (int b = 0; b < BD; ++b) {
        const int d = min(d0 + b, a.nd - 1);
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int e = tid + q * kThreads;
          if (e < PL) D[d * PL + e] = w[b][q];
        }
      }
    }
  }
  __syncthreads();

  // Flux sum of a moment at staged position p from the staged planes of the
  // other parity: x terms, then y terms, each in row order.
  auto flux = [&](const MomentRec& r, cptr<C> cf, int p) {
    C W = C(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = pick(r.jx, i) + p;
      W = couple(W, cf[i], to_c(L[q + 1]), to_c(L[q]));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = pick(r.jy, i) + p;
      W = couple(W, cf[4 + i], to_c(L[q + W2]), to_c(L[q]));
    }
    return W;
  };

  // Updates of G moments (records q0 .. q0 + G - 1, clamped to qend - 1: a
  // repeated record recomputes and rewrites the same value) at staged
  // position p standing for grid offsets co.  All reads of the group come
  // before its writes; a moment's update reads only the other parity and its
  // own old value, so the groups of one parity are independent.  Decay factors
  // are cached per grid of the parity (slot: cell centred along x or not).
  auto update_group = [&](int q0, int qend, int p, const ClassOffsets& co, C tau, DecayCache<C>& dc) {
    MomentRec r[G];
    C W[G], u[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int q = min(q0 + g, qend - 1);
      r[g] = moment_rec(tab, q);
      W[g] = flux(r[g], cat(coef, uint32_t(q) * uint32_t(8 * sizeof(C))), p);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) u[g] = to_c(L[r[g].n.z + p]);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint32_t off = co.of(r[g].g.x, r[g].g.y);
      if (r[g].g.w >= 0) W[g] += to_c(plane_at(src, r[g].g.w, ps)[off]);
      const bool s0 = r[g].g.x == 1;
      if (r[g].n.y) {
        const C c = D[r[g].g.z * PL + p];
        dc.set(s0, c, expm1div(-c * tau));
      }
      u[g] = sub_step(u[g], W[g], dc.c(s0), dc.e(s0), tau);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) L[r[g].n.z + p] = S(to_c(from_c<T>(u[g])));  // rounded to the storage type
  };

  // 2. odd moments on the tile and its ring (two positions per thread; a
  //    wave with no position in the second skips it)
  {
    const int e1 = tid + kThreads;
    const bool has1 = e1 < RN;
    const int ea = tid, eb = has1 ? e1 : 0;
    const int pa = (ea / RW + 1) * W2 + ea % RW + 1, pb = (eb / RW + 1) * W2 + eb % RW + 1;
    const ClassOffsets ca = class_offsets(x0 + ea % RW - 1, y0 + ea / RW - 1, a);
    const ClassOffsets cb = class_offsets(x0 + eb % RW - 1, y0 + eb / RW - 1, a);
    DecayCache<C> da{}, db{};
    for (int q0 = 0; q0 < a.nodd; q0 += G) {
      update_group(q0, a.nodd, pa, ca, a.tau_odd, da);
      if (has1) update_group(q0, a.nodd, pb, cb, a.tau_odd, db);
    }
  }
  __syncthreads();
  // 3. ring positions outside the grid on an extrapolation axis take the
  //    value of the grid point they repeat; the odd moments sit on two grid
  //    classes (cell centred along x or along y), so each ring position has
  //    one source per class, found once
  if (!a.px || !a.py) {
    int dst[2], src_x[2], src_y[2];  // per ring slot; source -1: no fix-up
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int e = tid + t * kThreads;
      const int lx = e % RW - 1, ly = e / RW - 1;
      dst[t] = (ly + 2) * W2 + lx + 2;
      src_x[t] = src_y[t] = -1;
      if (e < RN) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {  // c = 0: cell centred along x (nodal y); 1: along y
          const int mx = a.px ? lx : map_axis(x0 + lx, a.nx, 0, c == 0) - x0;
          const int my = a.py ? ly : map_axis(y0 + ly, a.ny, 0, c == 1) - y0;
          const int sidx = (mx != lx || my != ly) ? (my + 2) * W2 + mx + 2 : -1;
          if (c == 0)
            src_x[t] = sidx;
          else
            src_y[t] = sidx;
        }
      }
    }
    for (int q = 0; q < a.nodd; ++q) {
      const int4 g = rec4(tab, 4 * q);
      const int base = rec4(tab, 4 * q + 1).z;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int sidx = g.x == 1 ? src_x[t] : src_y[t];
        if (sidx >= 0) L[base + dst[t]] = L[base + sidx];
      }
    }
    __syncthreads();
  }

  // 4. even moments on the tile (one point per thread)
  const int tx = tid % TX, ty = tid / TX;
  const int pt = (ty + 2) * W2 + tx + 2;
  {
    const ClassOffsets ct = class_offsets(x0 + tx, y0 + ty, a);
    DecayCache<C> dt{};
    for (int q0 = a.nodd; q0 < a.nmom; q0 += G) update_group(q0, a.nmom, pt, ct, a.tau_even, dt);
  }
  __syncthreads();

  // 5. every moment's tile points that exist on its grid
  {
    const int X = x0 + tx, Y = y0 + ty;
    const bool in_x0 = X < a.nx + 1 - a.px, in_x1 = X < a.nx, in_y0 = Y < a.ny + 1 - a.py, in_y1 = Y < a.ny;
    const uint32_t off = uint32_t(Y * a.pitch + X);
#pragma unroll 4
    for (int q = 0; q < a.nmom; ++q) {
      const int4 g = rec4(tab, 4 * q);
      const int k = rec4(tab, 4 * q + 1).x;
      if ((g.x == 1 ? in_x1 : in_x0) && (g.y == 1 ? in_y1 : in_y0)) plane_at(uout, k, ps)[off] = from_c<T>(to_c(L[k * PL + pt]));
    }
  }
}

template <typename T>
size_t lds_t(int nmom, int nd) {
  using C = typename ComputeOf<T>::type;
  return size_t(nmom) * kFusedPlane * sizeof(typename StagedOf<T>::type) + size_t(nd) * kFusedPlane * sizeof(C);
}

template <typename T, int B>
hipError_t launch_b(const FusedArgs& f, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  const size_t lds = lds_t<T>(f.nmom, f.nd);
  static size_t attr = 0;  // per kernel instance
  if (lds > attr) {
    int dev = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    if (lds > size_t(max_lds)) return hipErrorInvalidValue;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&fused_kernel<T, kFusedTX, kFusedTY, B>),
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
  sc.nd = f.nd;
  sc.tau_odd = C(f.tau_odd);
  sc.tau_even = C(f.tau_even);
  hipLaunchKernelGGL((fused_kernel<T, kFusedTX, kFusedTY, B>), dim3(f.ntx * f.nty), dim3(kThreads), lds, stream,
                     static_cast<const T*>(f.uin), static_cast<T*>(f.uout), static_cast<const T*>(f.src),
                     static_cast<const C*>(f.decay), f.tab, static_cast<const C*>(f.coef), sc);
  return hipGetLastError();
}

// Staging batch: the smallest of 12, 24, 36 planes that holds every moment
// (36 = (N + 1)(N + 2) / 2 at N = 7).
template <typename T>
hipError_t launch_t(const FusedArgs& f, hipStream_t stream) {
  if (f.nmom <= 12) return launch_b<T, 12>(f, stream);
  if (f.nmom <= 24) return launch_b<T, 24>(f, stream);
  if (f.nmom <= 36) return launch_b<T, 36>(f, stream);
  return hipErrorInvalidValue;
}

}  // namespace

size_t fused_lds_bytes(int storage, int nmom, int nd) {
  switch (storage) {
    case STORE_FP64: return lds_t<double>(nmom, nd);
    case STORE_FP32: return lds_t<float>(nmom, nd);
    case STORE_BF16: return lds_t<bf16>(nmom, nd);
  }
  return 0;
}

hipError_t launch_fused(int storage, const FusedArgs& f, hipStream_t stream) {
  if (f.nmom < 1 || f.nodd < 0 || f.nodd > f.nmom || f.nd < 1 || f.ntx < 1 || f.nty < 1) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return launch_t<double>(f, stream);
    case STORE_FP32: return launch_t<float>(f, stream);
    case STORE_BF16: return launch_t<bf16>(f, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace starmap
