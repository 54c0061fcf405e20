// Device helpers shared by the kernels of the library: storage types, the
// compute type of each, bfloat16 rounding, boundary index maps and the
// XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace starmap {

struct bf16 {
  uint16_t bits;
};

template <typename T> struct ComputeOf { using type = float; };
template <> struct ComputeOf<double> { using type = double; };

__device__ __forceinline__ double to_c(double v) { return v; }
__device__ __forceinline__ float to_c(float v) { return v; }
__device__ __forceinline__ float to_c(bf16 v) { return __uint_as_float(uint32_t(v.bits) << 16); }

// Type of a staged LDS window: the storage type, except that BF16 values are
// widened to FP32 when staged (16-bit LDS accesses cannot be paired and their
// writes share dwords; the widening is exact).
template <typename T>
struct StagedOf {
  using type = T;
};
template <>
struct StagedOf<bf16> {
  using type = float;
};

template <typename T> __device__ __forceinline__ T from_c(typename ComputeOf<T>::type v);
template <> __device__ __forceinline__ double from_c<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_c<float>(float v) { return v; }
template <> __device__ __forceinline__ bf16 from_c<bf16>(float v) {
  // round to nearest even (the hardware conversion); NaN stays NaN
  return bf16{__builtin_bit_cast(uint16_t, static_cast<__bf16>(v))};
}

__device__ __forceinline__ double expm1_c(double z) { return expm1(z); }
__device__ __forceinline__ float expm1_c(float z) { return expm1f(z); }

// E(z) = (e^z - 1) / z with E(0) = 1.
template <typename C>
__device__ __forceinline__ C expm1div(C z) {
  return z == C(0) ? C(1) : expm1_c(z) / z;
}

// The two pieces of arithmetic of an update, with their fused multiply-adds
// spelled out so that every kernel that applies them (the separate sweeps,
// the batched sweep, the parity-fused pass) rounds identically:
// one coupling term of the residual, W + cf (hi - lo), and the exact sub-step
// u + tau (W - c u) E.
template <typename C>
__device__ __forceinline__ C couple(C W, C cf, C hi, C lo) {
  return fma(cf, hi - lo, W);
}
template <typename C>
__device__ __forceinline__ C sub_step(C u, C W, C c, C E, C tau) {
  return fma(tau * fma(-c, u, W), E, u);
}

// Index of an LDS staging load along one axis: periodic grids wrap, the others
// clamp to the last stored point (the constant-extrapolation ghosts of cell
// grids are exactly the clamped neighbours; clamped nodal points beyond the
// grid only feed outputs that are not stored).
__device__ __forceinline__ int map_axis(int i, int n, int periodic, int is_cell) {
  if (periodic) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  const int last = is_cell ? n - 1 : n;
  return i < 0 ? 0 : (i > last ? last : i);
}

// Blocks are dispatched round-robin over the 8 XCDs; hand each XCD a
// contiguous range of tiles so the halos of neighbouring tiles hit its L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int q = nblocks / 8, r = nblocks % 8;
  const int xcd = b % 8, idx = b / 8;
  // XCD x owns tiles [start(x), start(x) + q + (x < r))
  const int start = xcd * q + (xcd < r ? xcd : r);
  return start + idx;
}

// Tile number t -> tile column and row.  strip >= 2: tiles are numbered in
// strips of `strip` tile rows, and within a strip column by column:
// consecutive tiles are vertical neighbours (they share a halo row) and
// horizontal neighbours are `strip` tiles apart.  strip <= -2: strips of
// -strip tile columns, row by row within a strip: consecutive tiles are
// horizontal neighbours (they share a halo column) and vertical neighbours
// are -strip tiles apart.  Otherwise the tiles are numbered row by row.
// With the XCD-contiguous block order, tiles a few numbers apart run at
// nearly the same time on one XCD and can share halo lines in its L2.
__device__ __forceinline__ int2 tile_xy(int t, int ntx, int nty, int strip) {
  if (strip >= 2) {
    const int band = t / (strip * ntx);
    const int row0 = band * strip;
    const int rows = min(strip, nty - row0);
    const int r = t - band * strip * ntx;
    return make_int2(r / rows, row0 + r % rows);
  }
  if (strip <= -2) {
    const int w = -strip;
    const int band = t / (w * nty);
    const int col0 = band * w;
    const int cols = min(w, ntx - col0);
    const int r = t - band * w * nty;
    return make_int2(col0 + r % cols, r / cols);
  }
  return make_int2(t % ntx, t / ntx);
}

// Kernel tables (sweep programs, coupling records) are read-only during a
// launch and read at wave-uniform addresses: held as
// constant-address-space pointers, those reads are scalar loads wherever the
// pointer comes from (a kernel argument or an instance table in memory).
template <typename P>
using cptr = __attribute__((address_space(4))) const P*;

// Plane k of an array of planes of ps elements: a 32 x 32 -> 64-bit product
// (plane strides and plane counts fit 32 bits), cheaper in scalar
// instructions than a 64-bit multiply.
template <typename P>
__device__ __forceinline__ P* plane_at(P* base, int k, uint32_t ps) {
  return base + uint64_t(uint32_t(k)) * uint64_t(ps);
}

// Table entry at a 32-bit byte offset (non-negative indices): the scalar load
// takes the offset as its own operand, with no 64-bit address arithmetic.
template <typename P>
__device__ __forceinline__ cptr<P> cat(cptr<P> t, uint32_t byte_off) {
  return reinterpret_cast<cptr<P>>(reinterpret_cast<cptr<char>>(t) + byte_off);
}

// Entry i of a table of int4 records.
__device__ __forceinline__ int4 rec4(cptr<int> t, int i) {
  const cptr<int> q = cat(t, uint32_t(i) * 16u);
  return make_int4(q[0], q[1], q[2], q[3]);
}

}  // namespace starmap
