// Parity sweep of the staggered-grid P_N scheme on gfx950.
//
// One sweep applies the half-step operator S^p_tau of one parity p
// (Seibold & Frank, Sect. 4.3, eqs. solution_operator_even/_odd): for every
// component k of parity p and every point of its grid,
//   W_k = - sum_j Mx(k,j) D_x u_j - sum_j My(k,j) D_y u_j      (other parity j)
//   u_k <- u_k + tau (W_k + q_k - c_k u_k) E(-c_k tau),  E(z) = (e^z - 1)/z.
//
// Work decomposition: the outputs of a sweep are split into ranges of the
// azimuthal index m (an output (l, m) couples only to inputs (l -+ 1, m -+ 1),
// Lemma 2).  One workgroup of 256 threads handles one spatial tile of TX x TY
// points and one m range, walking the output orders from the top down.  For
// output order l it needs the input orders l + 1 and l - 1 inside the m range,
// staged in LDS as (TX+1) x (TY+1) tiles (one halo column and row, on the low
// side for cell-centred inputs and the high side for nodal ones); order l - 1
// stays staged for output order l - 2, and while one order is computed the
// next order's planes and output rows are already loading into registers.
// Every staged value feeds up to eight coupled outputs.  Boundary conditions
// enter only through the index mapping of the staging loads (wrap for
// periodic, clamp for extrapolation), so the stencil itself is uniform.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"

namespace starmap {

// Scalars of a sweep; the pointers travel as separate __restrict__ kernel
// arguments so the compiler may read the (uniform) program tables through the
// scalar cache while the state is written.
template <typename C>
struct SweepScalars {
  uint32_t ps;  // plane stride in elements
  int pitch, nx, ny, px, py, ntx, nty, nchunks, zero_off, parity, strip;
  C tau;
};

// Output values are written once per sweep and not read again before the
// next sweep: stream them past the caches.
__device__ __forceinline__ void store_stream(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void store_stream(bf16* p, bf16 v) {
  __builtin_nontemporal_store(v.bits, reinterpret_cast<uint16_t*>(p));
}

// Element at a 32-bit byte offset from a wave-uniform base: the address is
// base + zero-extended offset, which the compiler issues as a global access
// with a scalar base and one VGPR offset (no 64-bit address arithmetic).
template <typename T>
__device__ __forceinline__ T* at(T* base, uint32_t byte_off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ const T* at(const T* base, uint32_t byte_off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}

// A stored value as raw bits for a register: BF16 as its 16 bits in the low
// half of a 32-bit value (widened where it is used), other types as they are.
// The _stream forms read output rows, which are read once per sweep, just
// before they are overwritten.
__device__ __forceinline__ uint32_t load_raw(const bf16* p) { return *reinterpret_cast<const uint16_t*>(p); }
__device__ __forceinline__ float load_raw(const float* p) { return *p; }
__device__ __forceinline__ double load_raw(const double* p) { return *p; }
__device__ __forceinline__ uint32_t load_raw_stream(const bf16* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const uint16_t*>(p));
}
__device__ __forceinline__ float load_raw_stream(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ double load_raw_stream(const double* p) { return __builtin_nontemporal_load(p); }

// Two x-adjacent bfloat16 values as one 32-bit access (4-byte aligned).
__device__ __forceinline__ uint32_t load_pair_stream(const bf16* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const uint32_t*>(p));
}
__device__ __forceinline__ void store_pair_stream(bf16* p, bf16 lo, bf16 hi) {
  __builtin_nontemporal_store(uint32_t(lo.bits) | (uint32_t(hi.bits) << 16), reinterpret_cast<uint32_t*>(p));
}
// Two x-adjacent FP32 values as one 8-byte access (8-byte aligned).
typedef float float2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2v load_pair2_stream(const float* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const float2v*>(p));
}
__device__ __forceinline__ void store_pair_stream(float* p, float lo, float hi) {
  const float2v v = {lo, hi};
  __builtin_nontemporal_store(v, reinterpret_cast<float2v*>(p));
}
// (never called for the other storage types)
template <typename T>
__device__ __forceinline__ float2v load_pair2_stream(const T*) { return float2v{0.f, 0.f}; }
template <typename T>
__device__ __forceinline__ uint32_t load_pair_stream(const T*) { return 0; }
template <typename T>
__device__ __forceinline__ void store_pair_stream(T*, T, T) {}

// s_waitcnt immediate for vmcnt(0) with the other counters left alone
// (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int kWaitVm0 = 0x0F70;

// BF16 and FP32 on tiles of 512 points: each thread owns two x-adjacent
// output points, and on tiles away from the right edge of the grid (where no
// staging index is clamped or wrapped) the pair moves as one 32-bit (FP32:
// 64-bit) access: single accesses would move half the bytes per instruction.
template <typename T, int TX, int TY>
constexpr bool kPair = TX * TY == 512 && (sizeof(T) == 2 || sizeof(T) == 4);
// FP64 and FP32 on tiles of 256 points, FP32 and BF16 on tiles of 512,
// whose halo fits 128 threads: the window is staged by two halves of the
// workgroup, each half taking every other plane, each thread two (512-point
// tiles: four) x-adjacent points of it with one load of 16 bytes (FP32 on
// 256 points, BF16: 8) where they lie inside the grid: fewer vector memory
// instructions per staged plane than one point (BF16: one pair) per thread.
template <typename T, int TX, int TY>
constexpr bool kWide = (sizeof(T) == 8 ? TX * TY == 256 && TX % 2 == 0
                        : sizeof(T) == 4 ? (TX * TY == 256 && TX % 2 == 0) || (TX * TY == 512 && TX % 4 == 0)
                                         : TX * TY == 512 && TX % 4 == 0) &&
                       TX + TY <= 128;

// Whether work item lb lies on a tile whose pairs all lie inside the grid
// along x (FAST = true below); uniform over the workgroup.
template <typename T, int TX, int TY, typename C>
__device__ __forceinline__ bool pair_fast(const SweepScalars<C>& a, int lb) {
  if constexpr (!kPair<T, TX, TY> && !kWide<T, TX, TY>) {
    return false;
  } else {
    const int2 txy = tile_xy(lb / a.nchunks, a.ntx, a.nty, a.strip);
    return txy.x * TX + TX <= a.nx;
  }
}

// Body of one workgroup's work in a sweep: spatial tile and m range number lb
// (lb = tile * nchunks + range) of one instance.  FAST (pair tiles away from
// the grid's right edge) is a template argument, so the pair and the single
// accesses are separate code and no load sits under a branch on it.
template <typename T, int TX, int TY, int CAP, bool FAST>
__device__ __forceinline__ void sweep_tile(T* __restrict__ U, const typename ComputeOf<T>::type* __restrict__ decay,
                                           cptr<int> chunks, cptr<int> orders, cptr<int> loads, cptr<int> rows,
                                           cptr<typename ComputeOf<T>::type> rcoef,
                                           const SweepScalars<typename ComputeOf<T>::type>& a, const int lb) {
  using C = typename ComputeOf<T>::type;
  using S = typename StagedOf<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  S* L = reinterpret_cast<S*>(smem);
  constexpr int LW = TX + 1;
  constexpr int P = (TX + 1) * (TY + 1);
  constexpr int NP = TX * TY;
  static_assert(NP == 256 || NP == 512, "tile must hold 256 or 512 points");
  static_assert(TX + TY <= 256, "halo points must fit one per thread");
  constexpr int PPT = NP / 256;  // output points per thread
  constexpr int NG = 1;          // every thread owns its own points
  // Pipeline: while window o is computed, the planes of window o+1 (up to CAP)
  // and the first RB output rows of order o+1 are loaded into registers.
  constexpr int MAXP = CAP;
  constexpr int RB = CAP - 2;  // an m range of width w has w rows and w + 2 staged planes per order
  constexpr int LB = sizeof(T) >= 8 ? 8 : 16;  // planes per batch of the synchronous staging
  constexpr bool PAIR = kPair<T, TX, TY>;
  constexpr bool WIDE = kWide<T, TX, TY>;
  static_assert(PAIR || WIDE || !FAST, "the fast paths are for pair tiles (512 points) and wide staging");
  constexpr int SE = WIDE ? NP / 128 : PPT;  // staged interior points per thread and plane
  constexpr int EPT = SE + 1;           // staged points per thread and plane: interior + halo
  constexpr int SP = WIDE ? 2 : 1;      // thread halves that take turns in the planes of a window
  static_assert(MAXP % SP == 0 && LB % SP == 0, "planes split evenly over the thread halves");
  // BF16 values travel from memory to their first use as raw bit patterns
  // (16 bits in the low half of a register, or a pair as one 32-bit word):
  // widening them right after the load would be an immediate use of the load,
  // and its wait would hold the next order's prefetch behind the current one
  using RW = std::conditional_t<sizeof(T) == 2, uint32_t, T>;

  const int tid = threadIdx.x;
  // staging thread index and half (WIDE: threads 0-127 stage planes 0, 2, ...
  // of a window, threads 128-255 planes 1, 3, ...)
  const int st = WIDE ? (tid & 127) : tid;
  const int half = WIDE ? __builtin_amdgcn_readfirstlane(tid >> 7) : 0;
  const int tile = lb / a.nchunks;
  const int4 chk = rec4(chunks, lb - tile * a.nchunks);
  if (chk.x >= chk.y) return;  // no output rows in this m range
  const int2 txy = tile_xy(tile, a.ntx, a.nty, a.strip);
  const int x0 = txy.x * TX;
  const int y0 = txy.y * TY;
  const int grp = 0;
  constexpr bool pfast = FAST;  // every interior index of the tile maps to itself

  // Staging of one input plane into its (TX+1) x (TY+1) LDS tile.  The tile
  // holds global points (x0 - ox + lx, y0 - oy + ly), with ox (oy) = 1 for an
  // input cell-centred along x (y).  Staging thread t loads SE interior
  // points, x-adjacent on pair and wide tiles (a wave reads whole aligned
  // row segments; they need not be the points t updates) and, for
  // t < TY + TX, one halo point: of the halo column read by x differences
  // (lx = 0 or TX) or of the halo row read by y differences (ly = 0 or TY);
  // the corners are never read.  Source and LDS offsets are affine in (ox, oy):
  // src = sb + ox * sx + oy * sy, dst = db + ox * ddx + oy * ddy.  ox and oy
  // are 0 or 1 and uniform, so they enter as masks (no integer multiplies);
  // source offsets are 32-bit byte offsets from the plane base (sums wrap
  // modulo 2^32 to the in-plane offset).
  uint32_t sb[EPT], sx[EPT], sy[EPT];
  int db[EPT], ddx[EPT], ddy[EPT];
  constexpr uint32_t TS = sizeof(T);
  bool sv[EPT];
#pragma unroll
  for (int p = 0; p < SE; ++p) {
    const int e = WIDE ? SE * st + p : PAIR ? 2 * st + p : tid + p * 256;
    const int tx = e % TX, ty = e / TX;
    const int xn = map_axis(x0 + tx, a.nx, a.px, 0), xc = map_axis(x0 + tx, a.nx, a.px, 1);
    const int yn = map_axis(y0 + ty, a.ny, a.py, 0), yc = map_axis(y0 + ty, a.ny, a.py, 1);
    sb[p] = uint32_t(yn * a.pitch + xn) * TS;
    sx[p] = uint32_t(xc - xn) * TS;
    sy[p] = uint32_t((yc - yn) * a.pitch) * TS;
    db[p] = ty * LW + tx;
    ddx[p] = 1;
    ddy[p] = LW;
    sv[p] = true;
  }
  {
    constexpr int h = SE;
    sv[h] = st < TY + TX;
    if (st < TY) {  // halo column, row i
      const int i = st;
      const int xn = map_axis(x0 + TX, a.nx, a.px, 0), xc = map_axis(x0 - 1, a.nx, a.px, 1);
      const int yn = map_axis(y0 + i, a.ny, a.py, 0), yc = map_axis(y0 + i, a.ny, a.py, 1);
      sb[h] = uint32_t(yn * a.pitch + xn) * TS;
      sx[h] = uint32_t(xc - xn) * TS;
      sy[h] = uint32_t((yc - yn) * a.pitch) * TS;
      db[h] = i * LW + TX;
      ddx[h] = -TX;
      ddy[h] = LW;
    } else {  // halo row, column j (lanes past the halo keep in-bounds values)
      const int j = st < TY + TX ? st - TY : 0;
      const int xn = map_axis(x0 + j, a.nx, a.px, 0), xc = map_axis(x0 + j, a.nx, a.px, 1);
      const int yn = map_axis(y0 + TY, a.ny, a.py, 0), yc = map_axis(y0 - 1, a.ny, a.py, 1);
      sb[h] = uint32_t(yn * a.pitch + xn) * TS;
      sx[h] = uint32_t(xc - xn) * TS;
      sy[h] = uint32_t((yc - yn) * a.pitch) * TS;
      db[h] = TY * LW + j;
      ddx[h] = 1;
      ddy[h] = -TY * LW;
    }
  }

  // my output points: LDS position, plane offset, and whether the point exists
  // on each of the sweep's two output grids
  int pos[PPT];
  uint32_t goff[PPT];  // element offset in a plane
  bool val0[PPT], val1[PPT];
  {
    // even sweep: slot 0 = G11 (cell, cell), slot 1 = G22 (node, node);
    // odd sweep:  slot 0 = G21 (node, cell), slot 1 = G12 (cell, node)
    const int nxc = a.nx, nxn = a.nx + 1 - a.px, nyc = a.ny, nyn = a.ny + 1 - a.py;
    const int vx0 = a.parity ? nxn : nxc, vy0 = a.parity ? nyc : nyc;
    const int vx1 = a.parity ? nxc : nxn, vy1 = a.parity ? nyn : nyn;
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      int tx, ty;
      if constexpr (PAIR) {
        // each half-wave owns a 32 x 2 block of the tile, 16 lanes per row:
        // its stride-2 stencil reads of the LDS window (row pitch TX + 1,
        // an odd number of words) then meet each of the 32 banks once
        static_assert(TX % 32 == 0 && TY % 2 == 0, "pair tiles are made of 32 x 2 blocks");
        constexpr int CB = TX / 32;  // blocks per tile row
        const int u = tid >> 5;
        tx = (u % CB) * 32 + 2 * (tid & 15) + p;
        ty = 2 * (u / CB) + ((tid >> 4) & 1);
      } else {
        const int e = tid + p * 256;
        tx = e % TX;
        ty = e / TX;
      }
      const int X = x0 + tx, Y = y0 + ty;
      pos[p] = ty * LW + tx;
      goff[p] = uint32_t(Y * a.pitch + X);
      val0[p] = X < vx0 && Y < vy0;
      val1[p] = X < vx1 && Y < vy1;
    }
  }

  // the staged points of one input plane (load record ld) into registers
  // Only the waves holding halo threads (t < TX + TY) load halo points: the
  // others skip that load instruction (a wave-uniform branch), its value
  // would never reach the LDS.
  const bool halo_wave = __builtin_amdgcn_readfirstlane(st >> 6) * 64 < TX + TY;
  auto load_window = [&](RW (&v)[EPT], const int4 ld) {
    const T* src = plane_at(U, ld.x, a.ps);
    const uint32_t mx = 0u - uint32_t(ld.z), my = 0u - uint32_t(ld.w);
    if constexpr (WIDE && pfast) {
      // the points are contiguous and aligned to their total size (x a
      // multiple of SE, pitch and plane stride multiples of 64 elements)
      if constexpr (sizeof(T) == 2) {  // four BF16 values as two raw words
        const uint2 w = *reinterpret_cast<const uint2*>(at(src, sb[0] + (sx[0] & mx) + (sy[0] & my)));
        v[0] = w.x;
        v[1] = w.y;
      } else if constexpr (SE == 4) {  // four FP32 values
        const float4 w = *reinterpret_cast<const float4*>(at(src, sb[0] + (sx[0] & mx) + (sy[0] & my)));
        v[0] = w.x;
        v[1] = w.y;
        v[2] = w.z;
        v[3] = w.w;
      } else {
        using T2 = std::conditional_t<sizeof(T) == 8, double2, float2>;
        const T2 w = *reinterpret_cast<const T2*>(at(src, sb[0] + (sx[0] & mx) + (sy[0] & my)));
        v[0] = w.x;
        v[1] = w.y;
      }
    } else if constexpr (PAIR && pfast) {
      if constexpr (sizeof(T) == 2) {
        v[0] = *reinterpret_cast<const uint32_t*>(at(src, sb[0] + (sx[0] & mx) + (sy[0] & my)));
      } else {  // FP32 pair tiles too wide for the wide staging (128 x 4)
        const float2 w = *reinterpret_cast<const float2*>(at(src, sb[0] + (sx[0] & mx) + (sy[0] & my)));
        v[0] = w.x;
        v[1] = w.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < SE; ++q) v[q] = load_raw(at(src, sb[q] + (sx[q] & mx) + (sy[q] & my)));
    }
    if (halo_wave) v[EPT - 1] = load_raw(at(src, sb[EPT - 1] + (sx[EPT - 1] & mx) + (sy[EPT - 1] & my)));
  };
  // value of staged point q of a window's registers (BF16 interior points
  // on the fast tiles: packed two to a word, the lower x in the low half)
  auto wval = [&](const RW (&v)[EPT], int q) -> C {
    if constexpr (sizeof(T) == 2) {
      if constexpr ((PAIR || WIDE) && pfast) {
        if (q < SE) return __uint_as_float((q & 1) ? (v[q >> 1] & 0xFFFF0000u) : (v[q >> 1] << 16));
      }
      return __uint_as_float(v[q] << 16);
    } else {
      return v[q];
    }
  };

  // synchronous staging of planes [b0, b1) of a load list into LDS
  auto stage_sync = [&](int first, int b0, int b1) {
    for (int bb = b0; bb < b1; bb += LB) {
      constexpr int LH = LB / SP;  // planes of the batch per thread half
      RW v[LH][EPT];
      // the records first (clamped into the list: every scalar load is
      // unconditional, so they issue together), then the loads they describe
      int4 lr[LH];
#pragma unroll
      for (int b = 0; b < LH; ++b) lr[b] = rec4(loads, first + min(bb + SP * b + half, b1 - 1));
#pragma unroll
      for (int b = 0; b < LH; ++b)
        if (bb + SP * b + half < b1) load_window(v[b], lr[b]);
#pragma unroll
      for (int b = 0; b < LH; ++b) {
        if (bb + SP * b + half < b1) {
          // read again (a scalar cache hit) rather than kept live across the loads
          const int4 ld = rec4(loads, first + bb + SP * b + half);
#pragma unroll
          for (int q = 0; q < EPT; ++q)
            if (sv[q]) L[ld.y + db[q] + (ddx[q] & -ld.z) + (ddy[q] & -ld.w)] = S(wval(v[b], q));
        }
      }
      // Every load of the batch has been consumed.  As at the end of the
      // order loop, the compiler cannot match the conditional loads with
      // their conditional stores: without this wait it takes the batch's
      // registers as possibly still loading at the next batch and waits for
      // all outstanding loads before each of its loads, one memory round
      // trip per plane.
      __builtin_amdgcn_s_waitcnt(kWaitVm0);
    }
  };

  // current values of the output rows r0, r0 + NG, ... (RB of them, < r1),
  // raw (a BF16 pair: one word in uv[i][0])
  auto load_rows = [&](RW (&uv)[RB][PPT], int r0, int r1) {
    // plane and grid slot of every row first (row indices clamped into the
    // table: unconditional scalar loads that issue together), then the loads
    int rk[RB], rs[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = __builtin_amdgcn_readfirstlane(max(min(r0 + NG * i, r1 - 1), 0));
      const cptr<int> rec = cat(rows, uint32_t(r) * 64u);
      rk[i] = rec[0];
      rs[i] = rec[1];
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int r = __builtin_amdgcn_readfirstlane(r0 + NG * i);
      if (r < r1) {
        const T* up = plane_at(U, rk[i], a.ps);
        const bool s1 = rs[i] != 0;
        if constexpr (PAIR && pfast && sizeof(T) == 2) {  // both points of the pair lie inside the output grid along x
          uint32_t w = 0;
          if (s1 ? val1[0] : val0[0]) w = load_pair_stream(at(up, goff[0] * TS));
          uv[i][0] = w;
        } else if constexpr (PAIR && pfast) {
          float2v w = {0.f, 0.f};
          if (s1 ? val1[0] : val0[0]) w = load_pair2_stream(at(up, goff[0] * TS));
          uv[i][0] = w.x;
          uv[i][1] = w.y;
        } else {
#pragma unroll
          for (int p = 0; p < PPT; ++p)
            uv[i][p] = (s1 ? val1[p] : val0[p]) ? load_raw_stream(at(up, goff[p] * TS)) : RW(0);
        }
      }
    }
  };
  // value of point p of a row's registers
  auto rval = [&](const RW (&uv)[PPT], int p) -> C {
    if constexpr (sizeof(T) == 2) {
      if constexpr (PAIR && pfast) return __uint_as_float(p == 0 ? (uv[0] << 16) : (uv[0] & 0xFFFF0000u));
      return __uint_as_float(uv[p] << 16);
    } else {
      return uv[p];
    }
  };

  // decay cache per output grid of the sweep: (plane id, c, E(-c tau))
  int cdk0 = -1, cdk1 = -1;
  C c0[PPT], e0[PPT], c1[PPT], e1[PPT];
  // The decay planes an order needs (one per output grid; they change with
  // the order when scattering or filtering is anisotropic) are loaded with
  // that order's window, so no load waits inside the compute.
  int ndk0 = -1, ndk1 = -1;
  C nc0[PPT], nc1[PPT];
  auto prefetch_decay = [&](const int4 od, C (&n0)[PPT], C (&n1)[PPT]) {
    // every row of an order shares the decay plane of its output grid
    ndk0 = -1;
    ndk1 = -1;
    for (int r = od.z + grp; r < od.w && (ndk0 < 0 || ndk1 < 0); r += NG) {
      const cptr<int> rr = cat(rows, uint32_t(r) * 64u);
      const int gs = rr[1], dk = rr[2];
      // value selects (a conditional store to one of two variables would be
      // merged into a store through a selected address, i.e. stack memory)
      ndk0 = (gs == 0 && ndk0 < 0) ? dk : ndk0;
      ndk1 = (gs != 0 && ndk1 < 0) ? dk : ndk1;
    }
    const bool l0 = ndk0 >= 0 && ndk0 != cdk0, l1 = ndk1 >= 0 && ndk1 != cdk1;
    const C* d0 = plane_at(decay, l0 ? ndk0 : 0, a.ps);
    const C* d1 = plane_at(decay, l1 ? ndk1 : 0, a.ps);
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      if (l0) n0[p] = val0[p] ? *at(d0, goff[p] * uint32_t(sizeof(C))) : C(0);
      if (l1) n1[p] = val1[p] ? *at(d1, goff[p] * uint32_t(sizeof(C))) : C(0);
    }
  };
  auto apply_decay = [&]() {
    if (ndk0 >= 0 && ndk0 != cdk0) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        c0[p] = nc0[p];
        e0[p] = expm1div(-nc0[p] * a.tau);
      }
      cdk0 = ndk0;
    }
    if (ndk1 >= 0 && ndk1 != cdk1) {
#pragma unroll
      for (int p = 0; p < PPT; ++p) {
        c1[p] = nc1[p];
        e1[p] = expm1div(-nc1[p] * a.tau);
      }
      cdk1 = ndk1;
    }
  };

  // the padding couplings read this plane of zeros
  for (int e = tid; e < P; e += 256) L[a.zero_off + e] = S(0);
  // prologue: the first rows and decay values, then the first window, so
  // that all of them are in flight together (one memory round trip; the
  // window's LDS stores wait for the window loads, issued last)
  RW ua[RB][PPT];
  {
    const int4 ord = rec4(orders, chk.x);
    load_rows(ua, ord.z + grp, ord.w);
    prefetch_decay(ord, nc0, nc1);
    stage_sync(ord.x, 0, ord.y - ord.x);
  }
  __builtin_amdgcn_s_waitcnt(kWaitVm0);  // see the end of the order loop
  __syncthreads();

  for (int o = chk.x; o < chk.y; ++o) {
    const int4 ord = rec4(orders, o);
    apply_decay();
    const bool has_next = o + 1 < chk.y;
    const int4 nxt = has_next ? rec4(orders, o + 1) : make_int4(0, 0, 0, 0);
    const int nl = nxt.y - nxt.x;
    // 1. the next window into registers (every thread loads its own elements)
    constexpr int MH = MAXP / SP;  // planes of the window per thread half
    RW stg[MH][EPT];
    {
      // the records first (clamped into the list: unconditional scalar loads
      // that issue together), then the loads they describe
      int4 nrec[MH];
#pragma unroll
      for (int b = 0; b < MH; ++b) nrec[b] = rec4(loads, nxt.x + max(min(SP * b + half, nl - 1), 0));
#pragma unroll
      for (int b = 0; b < MH; ++b)
        if (SP * b + half < nl) load_window(stg[b], nrec[b]);
    }
    // 2. the first output rows of the next order
    RW ub[RB][PPT];
    if (has_next) {
      load_rows(ub, nxt.z + grp, nxt.w);
      prefetch_decay(nxt, nc0, nc1);
    }
    // 3. update this order's rows from the current window
    for (int r0 = ord.z + grp; r0 < ord.w; r0 += NG * RB) {
      if (r0 != ord.z + grp) {  // more rows than the registers hold: load the next batch now
        load_rows(ua, r0, ord.w);
        __builtin_amdgcn_s_waitcnt(kWaitVm0);
      }
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const int r = __builtin_amdgcn_readfirstlane(r0 + NG * i);
        if (r < ord.w) {
          cptr<int> rec = cat(rows, uint32_t(r) * 64u);
          cptr<C> cf = cat(rcoef, uint32_t(r) * uint32_t(8 * sizeof(C)));
          const int k = rec[0], gslot = rec[1], so = rec[3];
          T* up = plane_at(U, k, a.ps);
          T nv[PPT];
#pragma unroll
          for (int p = 0; p < PPT; ++p) {
            C W = C(0);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const S* lp = L + rec[4 + t] + pos[p];
              W = couple(W, cf[t], to_c(lp[1]), to_c(lp[0]));
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const S* lp = L + rec[8 + t] + pos[p];
              W = couple(W, cf[4 + t], to_c(lp[LW]), to_c(lp[0]));
            }
    // the source, staged in LDS, joins the residual
            if (so >= 0) W += to_c(L[so + pos[p]]);
            const C c = gslot ? c1[p] : c0[p];
            const C E = gslot ? e1[p] : e0[p];
            nv[p] = from_c<T>(sub_step(rval(ua[i], p), W, c, E, a.tau));
            if (!(PAIR && pfast) && (gslot ? val1[p] : val0[p])) store_stream(at(up, goff[p] * TS), nv[p]);
          }
          if (PAIR && pfast && (gslot ? val1[0] : val0[0])) store_pair_stream(at(up, goff[0] * TS), nv[0], nv[PPT - 1]);
        }
      }
    }
    // 4. every read of the current window is done: install the next one
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MH; ++b) {
      if (SP * b + half < nl) {
        const int4 ld = rec4(loads, nxt.x + SP * b + half);
#pragma unroll
        for (int q = 0; q < EPT; ++q)
          if (sv[q]) L[ld.y + db[q] + (ddx[q] & -ld.z) + (ddy[q] & -ld.w)] = S(wval(stg[b], q));
      }
    }
    if (nl > MAXP) stage_sync(nxt.x, MAXP, nl);
    // Every load of this order has been consumed: wait for all of them here.
    // The compiler cannot match the conditional loads with their conditional
    // uses, so without this wait it assumes the window registers may still be
    // receiving and waits for every outstanding load at their first reuse,
    // which would stall the next order's prefetch right after it is issued.
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int p = 0; p < (PAIR && pfast && sizeof(T) == 2 ? 1 : PPT); ++p) ua[i][p] = ub[i][p];
  }
}

// Waves per SIMD the compiler is asked to fit (1: no bound).  The FP32
// 32 x 8 tile with eight planes in registers is held to seven: it needs two
// registers more than seven waves allow, and at m-range width 6 its LDS
// admits seven workgroups per CU.  (The batched kernel, which reads its
// instance table as well, would spill at that bound and keeps none.)
template <typename T, int TX, int TY, int CAP>
constexpr int kMinWaves = (sizeof(T) == 4 && TX == 32 && TY == 8 && CAP == 8) ? 7 : 1;

template <typename T, int TX, int TY, int CAP>
__global__ void __launch_bounds__(256, (kMinWaves<T, TX, TY, CAP>))
sweep_kernel(T* __restrict__ U, const typename ComputeOf<T>::type* __restrict__ decay,
             const int4* __restrict__ chunks, const int4* __restrict__ orders,
             const int4* __restrict__ loads, const int* __restrict__ rows,
             const typename ComputeOf<T>::type* __restrict__ rcoef,
             const SweepScalars<typename ComputeOf<T>::type> a) {
  // logical block = tile * nchunks + chunk: the m ranges of one tile run on
  // the same XCD, one after another, and share its L2
  using C = typename ComputeOf<T>::type;
  const int lb = xcd_tile(blockIdx.x, gridDim.x);
  if constexpr (kPair<T, TX, TY> || kWide<T, TX, TY>) {
    if (pair_fast<T, TX, TY>(a, lb)) {
      sweep_tile<T, TX, TY, CAP, true>(U, decay, (cptr<int>)chunks, (cptr<int>)orders, (cptr<int>)loads,
                                       (cptr<int>)rows, (cptr<C>)rcoef, a, lb);
      return;
    }
  }
  sweep_tile<T, TX, TY, CAP, false>(U, decay, (cptr<int>)chunks, (cptr<int>)orders, (cptr<int>)loads,
                                    (cptr<int>)rows, (cptr<C>)rcoef, a, lb);
}

// Sweep number j of a batched run.  Instances are sorted by their number of
// sweeps (descending), so the instances still running at sweep j are the
// first n_active; their workgroups (tiles x m ranges) are numbered
// consecutively, instance i owning [first[i], first[i+1]).  Sweep j has odd
// parity for even j (the composition starts and ends with odd half-steps).
// BatchEntry as the device reads it: pointers read from memory carry no
// address space, so without this the compiler would use flat accesses (which
// share the LDS wait counter) and vector loads for the uniform tables.
template <typename P>
using gptr = __attribute__((address_space(1))) P*;
struct BatchEntryG {
  gptr<void> u;
  gptr<const void> decay;
  gptr<const int4> chunks[2];
  gptr<const int4> orders[2];
  gptr<const int4> loads[2];
  gptr<const int> rows[2];
  gptr<const void> rcoef[2];
  int64_t plane_stride;
  double tau_full, tau_half;
  int pitch, nx, ny, px, py, ntx, nty, nchunks;
  int zero_off[2];
  int nsweeps;
  int strip;
  int64_t even_b_delta;
};
static_assert(sizeof(BatchEntryG) == sizeof(BatchEntry), "device view of BatchEntry");
static_assert(offsetof(BatchEntryG, even_b_delta) == offsetof(BatchEntry, even_b_delta), "device view of BatchEntry");
static_assert(offsetof(BatchEntryG, plane_stride) == offsetof(BatchEntry, plane_stride), "device view of BatchEntry");
static_assert(offsetof(BatchEntryG, nsweeps) == offsetof(BatchEntry, nsweeps), "device view of BatchEntry");

template <typename T, int TX, int TY, int CAP>
__global__ void __launch_bounds__(256)
sweep_batch_kernel(const BatchEntry* __restrict__ table, const int* __restrict__ first, const int n_active,
                   const int j) {
  using C = typename ComputeOf<T>::type;
  const int item = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = n_active - 1;  // last instance with first[i] <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= item) lo = mid; else hi = mid - 1;
  }
  const BatchEntryG& e = reinterpret_cast<const BatchEntryG*>(table)[lo];
  const int par = (j & 1) ? 0 : 1;
  // closure solvers: before even sweep j, (j + 1) / 2 odd sweeps have moved
  // the order-5 moments; an odd count leaves them in the closure planes
  const int64_t bd = (par == 0 && (((j + 1) >> 1) & 1)) ? e.even_b_delta : 0;
  SweepScalars<C> a;
  a.ps = uint32_t(e.plane_stride);
  a.pitch = e.pitch;
  a.nx = e.nx;
  a.ny = e.ny;
  a.px = e.px;
  a.py = e.py;
  a.ntx = e.ntx;
  a.nty = e.nty;
  a.nchunks = e.nchunks;
  a.zero_off = e.zero_off[par];
  a.parity = par;
  a.strip = e.strip;
  a.tau = C((j == 0 || j == e.nsweeps - 1) ? e.tau_half : e.tau_full);
  const int lb = item - first[lo];
  T* const u = (T*)(gptr<T>)e.u;
  const C* const dec = (const C*)(gptr<const C>)e.decay;
  const cptr<int> ch = (cptr<int>)((gptr<const char>)e.chunks[par] + bd);
  const cptr<int> od = (cptr<int>)((gptr<const char>)e.orders[par] + bd);
  const cptr<int> ldl = (cptr<int>)((gptr<const char>)e.loads[par] + bd);
  const cptr<int> rw = (cptr<int>)((gptr<const char>)e.rows[par] + bd);
  const cptr<C> rc = (cptr<C>)((gptr<const char>)e.rcoef[par] + bd);
  if constexpr (kPair<T, TX, TY> || kWide<T, TX, TY>) {
    if (pair_fast<T, TX, TY>(a, lb)) {
      sweep_tile<T, TX, TY, CAP, true>(u, dec, ch, od, ldl, rw, rc, a, lb);
      return;
    }
  }
  sweep_tile<T, TX, TY, CAP, false>(u, dec, ch, od, ldl, rw, rc, a, lb);
}

// ------------------------------------------------------------ variants
namespace {
// (tx, ty, cap): cap 10 holds the widest m range's planes of one order in
// registers; cap 8 and 6 hold fewer (the rest is staged synchronously) but
// leave registers for a fourth (fifth) workgroup per CU, which pays at the
// narrower m ranges
constexpr TileShape kVariants[] = {{64, 4, 10},  {128, 2, 10}, {32, 8, 10}, {32, 16, 10}, {128, 4, 10},
                                   {64, 8, 10},  {64, 8, 8},   {64, 8, 6},  {32, 8, 8},   {32, 8, 6},
                                   {64, 4, 8},   {32, 16, 8},  {128, 4, 8}, {64, 4, 6}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Opt the kernels of one instantiation in to all of the device's LDS (once).
template <typename T, int TX, int TY, int CAP>
hipError_t prepare_t(size_t lds) {
  static size_t attr_bytes = 0;
  if (lds <= attr_bytes) return hipSuccess;
  int dev = 0, max_lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  if (lds > size_t(max_lds)) return hipErrorInvalidValue;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sweep_kernel<T, TX, TY, CAP>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&sweep_batch_kernel<T, TX, TY, CAP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
  if (e != hipSuccess) return e;
  attr_bytes = size_t(max_lds);
  return hipSuccess;
}

template <typename T, int TX, int TY, int CAP>
size_t lds_t(int slots) {
  return size_t(slots) * (TX + 1) * (TY + 1) * sizeof(typename StagedOf<T>::type);
}

template <typename T, int TX, int TY, int CAP>
hipError_t launch_t(const void* args, int slots, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  const auto& a = *reinterpret_cast<const SweepArgs<C>*>(args);
  const size_t lds = lds_t<T, TX, TY, CAP>(slots);
  hipError_t e = prepare_t<T, TX, TY, CAP>(lds);
  if (e != hipSuccess) return e;
  SweepScalars<C> sc;
  sc.ps = uint32_t(a.plane_stride);
  sc.pitch = a.pitch;
  sc.nx = a.nx;
  sc.ny = a.ny;
  sc.px = a.px;
  sc.py = a.py;
  sc.ntx = a.ntx;
  sc.nty = a.nty;
  sc.nchunks = a.nchunks;
  sc.zero_off = a.zero_off;
  sc.parity = a.parity;
  sc.strip = a.strip;
  sc.tau = a.tau;
  const int blocks = a.ntx * a.nty * a.nchunks;
  hipLaunchKernelGGL((sweep_kernel<T, TX, TY, CAP>), dim3(blocks), dim3(256), lds, stream,
                     reinterpret_cast<T*>(a.u), a.decay, a.chunks, a.orders, a.loads, a.rows, a.rcoef, sc);
  return hipGetLastError();
}

template <typename T, int TX, int TY, int CAP>
hipError_t launch_batch_t(const BatchEntry* table, const int* first, int n_active, int items, int j, int slots,
                          hipStream_t stream) {
  const size_t lds = lds_t<T, TX, TY, CAP>(slots);
  hipError_t e = prepare_t<T, TX, TY, CAP>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((sweep_batch_kernel<T, TX, TY, CAP>), dim3(items), dim3(256), lds, stream, table, first,
                     n_active, j);
  return hipGetLastError();
}

// the compiled tile variants, in the order of kVariants
#define STARMAP_FOR_VARIANT(v, CALL)      \
  switch (v) {                            \
    case 0: return CALL(64, 4, 10);       \
    case 1: return CALL(128, 2, 10);      \
    case 2: return CALL(32, 8, 10);       \
    case 3: return CALL(32, 16, 10);      \
    case 4: return CALL(128, 4, 10);      \
    case 5: return CALL(64, 8, 10);       \
    case 6: return CALL(64, 8, 8);        \
    case 7: return CALL(64, 8, 6);        \
    case 8: return CALL(32, 8, 8);        \
    case 9: return CALL(32, 8, 6);        \
    case 10: return CALL(64, 4, 8);       \
    case 11: return CALL(32, 16, 8);      \
    case 12: return CALL(128, 4, 8);      \
    case 13: return CALL(64, 4, 6);       \
  }                                       \
  return hipErrorInvalidValue;

template <typename T>
hipError_t launch_typed(int variant, const void* args, int slots, hipStream_t stream) {
#define STARMAP_CALL(X, Y, K) launch_t<T, X, Y, K>(args, slots, stream)
  STARMAP_FOR_VARIANT(variant, STARMAP_CALL)
#undef STARMAP_CALL
}

template <typename T>
hipError_t launch_batch_typed(int variant, const BatchEntry* table, const int* first, int n_active, int items,
                              int j, int slots, hipStream_t stream) {
#define STARMAP_CALL(X, Y, K) launch_batch_t<T, X, Y, K>(table, first, n_active, items, j, slots, stream)
  STARMAP_FOR_VARIANT(variant, STARMAP_CALL)
#undef STARMAP_CALL
}

template <typename T>
hipError_t prepare_typed(int variant, int slots) {
#define STARMAP_CALL(X, Y, K) prepare_t<T, X, Y, K>(lds_t<T, X, Y, K>(slots))
  STARMAP_FOR_VARIANT(variant, STARMAP_CALL)
#undef STARMAP_CALL
}
#undef STARMAP_FOR_VARIANT
}  // namespace

int sweep_variant_count() { return kNumVariants; }
TileShape sweep_variant(int v) { return kVariants[v]; }


size_t sweep_lds_bytes(int v, int slots, int storage) {
  const size_t s = storage == STORE_FP64 ? 8 : 4;  // BF16 windows are staged as FP32
  return size_t(slots) * (kVariants[v].tx + 1) * (kVariants[v].ty + 1) * s;
}

hipError_t prepare_sweep(int storage, int variant, int slots) {
  if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return prepare_typed<double>(variant, slots);
    case STORE_FP32: return prepare_typed<float>(variant, slots);
    case STORE_BF16: return prepare_typed<bf16>(variant, slots);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_batch(int storage, int variant, const BatchEntry* table, const int* first, int n_active,
                              int items, int j, int slots, hipStream_t stream) {
  if (variant < 0 || variant >= kNumVariants || n_active < 1 || items < 1) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return launch_batch_typed<double>(variant, table, first, n_active, items, j, slots, stream);
    case STORE_FP32: return launch_batch_typed<float>(variant, table, first, n_active, items, j, slots, stream);
    case STORE_BF16: return launch_batch_typed<bf16>(variant, table, first, n_active, items, j, slots, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(int storage, int variant, const void* args, int slots, hipStream_t stream) {
  if (variant < 0 || variant >= kNumVariants) return hipErrorInvalidValue;
  switch (storage) {
    case STORE_FP64: return launch_typed<double>(variant, args, slots, stream);
    case STORE_FP32: return launch_typed<float>(variant, args, slots, stream);
    case STORE_BF16: return launch_typed<bf16>(variant, args, slots, stream);
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ diagnostics
// Block partials in FP64, then one block sums them in a fixed order, so the
// result does not depend on scheduling.
template <typename T>
__global__ void __launch_bounds__(256) diag_partial_kernel(DiagArgs a) {
  __shared__ double s_sum[256], s_sq[256], s_max[256], s_bad[256];
  const int plane = blockIdx.x / a.blocks_per_plane;
  const int rb = blockIdx.x % a.blocks_per_plane;
  const int nxp = a.plane_nx[plane], nyp = a.plane_ny[plane];
  const int r0 = rb * a.rows_per_block;
  const int r1 = min(nyp, r0 + a.rows_per_block);
  const T* U = reinterpret_cast<const T*>(a.u) + int64_t(plane) * a.plane_stride;
  double sum = 0.0, sq = 0.0, mx = 0.0, bad = 0.0;
  for (int r = r0; r < r1; ++r) {
    for (int x = threadIdx.x; x < nxp; x += 256) {
      const double v = double(to_c(U[int64_t(r) * a.pitch + x]));
      if (!isfinite(v)) { bad += 1.0; continue; }
      sum += v;
      sq += v * v;
      mx = fmax(mx, fabs(v));
    }
  }
  s_sum[threadIdx.x] = sum;
  s_sq[threadIdx.x] = sq;
  s_max[threadIdx.x] = mx;
  s_bad[threadIdx.x] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
      s_sq[threadIdx.x] += s_sq[threadIdx.x + w];
      s_max[threadIdx.x] = fmax(s_max[threadIdx.x], s_max[threadIdx.x + w]);
      s_bad[threadIdx.x] += s_bad[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* p = a.part + 4 * int64_t(blockIdx.x);
    p[0] = plane == 0 ? s_sum[0] : 0.0;
    p[1] = s_sq[0];
    p[2] = s_max[0];
    p[3] = s_bad[0];
  }
}

__global__ void __launch_bounds__(256) diag_final_kernel(const double* part, int nblocks, double* out) {
  __shared__ double s[4][256];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) {
    a0 += part[4 * b + 0];
    a1 += part[4 * b + 1];
    a2 = fmax(a2, part[4 * b + 2]);
    a3 += part[4 * b + 3];
  }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  s[2][threadIdx.x] = a2;
  s[3][threadIdx.x] = a3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] += s[0][threadIdx.x + w];
      s[1][threadIdx.x] += s[1][threadIdx.x + w];
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
      s[3][threadIdx.x] += s[3][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

int diag_blocks(int nplanes, int max_rows, int rows_per_block) {
  return nplanes * ((max_rows + rows_per_block - 1) / rows_per_block);
}

hipError_t launch_diagnostics(int storage, const DiagArgs& a, hipStream_t stream) {
  const int nb = a.nplanes * a.blocks_per_plane;
  switch (storage) {
    case STORE_FP64: hipLaunchKernelGGL(diag_partial_kernel<double>, dim3(nb), dim3(256), 0, stream, a); break;
    case STORE_FP32: hipLaunchKernelGGL(diag_partial_kernel<float>, dim3(nb), dim3(256), 0, stream, a); break;
    case STORE_BF16: hipLaunchKernelGGL(diag_partial_kernel<bf16>, dim3(nb), dim3(256), 0, stream, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, stream, a.part, nb, a.out);
  return hipGetLastError();
}

}  // namespace starmap
