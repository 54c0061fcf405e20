// Device kernels of the staggered-grid P_N step and their launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace starmap {

enum StorageType : int { STORE_FP64 = 0, STORE_FP32 = 1, STORE_BF16 = 2 };

// Kernel arguments of one parity sweep (passed by value).
template <typename C>
struct SweepArgs {
  void* u;                 // state planes, then source planes, storage type
  const C* decay;          // decay planes c(x, y), compute type
  const int4* chunks;      // (order0, order1, -, -) per m range
  const int4* orders;      // (load0, load1, row0, row1) per output order
  const int4* loads;       // (k, lds offset, ox, oy)
  const int* rows;         // 16 ints per row: k, gslot, dk, source LDS offset, xo[4], yo[4], unused[4]
  const C* rcoef;          // 8 coefficients per row (x couplings, then y couplings)
  int64_t plane_stride;    // elements between consecutive planes
  int pitch;               // elements between rows
  int nx, ny, px, py;      // cells per axis, periodicity flags
  int ntx, nty;            // tiles per axis
  int nchunks;             // workgroups per tile (m ranges)
  int zero_off;            // LDS element offset of the zero plane
  int parity;              // 0: outputs on G11/G22, 1: outputs on G21/G12
  int strip;               // tile rows per strip of the tile order (<= 1: row by row)
  C tau;                   // sub-step length
};

struct TileShape {
  int tx, ty;
  int cap;  // planes of one staged order and output rows per order held in registers
};

// Tile shapes compiled into the library (index = variant id).
int sweep_variant_count();
TileShape sweep_variant(int v);

// LDS bytes a variant needs for slots planes of the given storage type.
size_t sweep_lds_bytes(int v, int slots, int storage);

// Launch one sweep; args.u etc. must be device pointers.  Returns a HIP error.
hipError_t launch_sweep(int storage, int variant, const void* args, int slots, hipStream_t stream);

// One instance of a batched run: device pointers of its state, decay planes
// and the sweep programs of both parities, and its scalars.
struct BatchEntry {
  void* u;
  const void* decay;  // compute type
  const int4* chunks[2];
  const int4* orders[2];
  const int4* loads[2];
  const int* rows[2];
  const void* rcoef[2];  // compute type
  int64_t plane_stride;
  double tau_full, tau_half;  // dt and dt / 2
  int pitch, nx, ny, px, py, ntx, nty, nchunks;
  int zero_off[2];
  int nsweeps;  // sweeps still to run: 2 n + 1 for n steps
  int strip;    // tile rows per strip of the tile order
  // closure solvers: bytes from the even sweep's program to the one that reads
  // the order-5 moments from the closure planes (0: none)
  int64_t even_b_delta;
};

// Opts the kernels of a variant in to the LDS it needs (outside any stream
// capture).  Returns a HIP error.
hipError_t prepare_sweep(int storage, int variant, int slots);

// Launch sweep number j of a batched run over the first n_active instances of
// table, whose workgroups are numbered from first[i]; items = first[n_active].
hipError_t launch_sweep_batch(int storage, int variant, const BatchEntry* table, const int* first, int n_active,
                              int items, int j, int slots, hipStream_t stream);

// Linear combination of basis planes (compute type) into decay planes
// (compute type) or source planes (storage type).  For each pair (o, d) of
// list: plane d of out = cst[o] + sum over entries e in [first[o], first[o+1])
// of sign_e * factor_e * basis[b_e], where entries holds (b_e, term_e, sign_e)
// and factor_e = a[term_e] (or 1 when term_e < 0).
constexpr int COMBINE_MAX_TERMS = 32;
struct CombineArgs {
  const void* basis;
  const int* first;
  const int* entries;
  const double* cst;  // per output: constant added to the sum
  const int* list;
  void* out;
  int64_t plane_stride;
  int nlist;
  double a[COMBINE_MAX_TERMS];
};
hipError_t launch_combine(int storage, bool to_compute_type, const CombineArgs& a, hipStream_t stream);

// Diffusion step of the D_N model on the order-N moments (j = 0..nplanes-1):
// tmp[j] = u_k + tau kappa_j (second difference along x * rdx2 + along y *
// rdy2) at every point of moment k's grid (tab[3j] = k, tab[3j+1] = gx,
// tab[3j+2] = gy), with the staging index map at the boundary; then the
// copy kernel writes tmp[j] back to plane k.
struct DiffusionArgs {
  void* u;            // state planes, storage type
  void* tmp;          // nplanes scratch planes, storage type
  const void* kappa;  // nplanes planes, compute type
  const int* tab;
  int64_t plane_stride;
  int pitch, nx, ny, px, py, nplanes;
  double rdx2, rdy2, tau;
};
hipError_t launch_diffusion(int storage, const DiffusionArgs& a, int max_points, hipStream_t stream);

// Parity-fused pass (small orders): S^o_tau_odd then S^e_tau_even on tiles of
// 32 x 8 points, all moments of a tile in LDS.  Reads uin (state planes),
// writes uout (another buffer of state planes); sources at src (plane
// tab[16k+3] of src, or none), decay planes at decay.  tab holds 16 ints per
// moment: grid classes gx, gy (1 = cell, 2 = node), decay plane, source plane
// or -1, number of x and y couplings, the coupled moments (4 + 4), unused;
// coef holds the 8 coupling coefficients of the separate sweeps' programs;
// order lists the odd moments (nodd of them), then the even ones.
template <typename C>
struct FusedScalars {
  uint32_t ps;
  int pitch, nx, ny, px, py, ntx, nty, nmom, nodd, nd;
  C tau_odd, tau_even;
};
// Tile of the parity-fused pass and its staged plane (two-point halo): the
// host's coupling table holds LDS offsets in these units.
constexpr int kFusedTX = 32, kFusedTY = 8;
constexpr int kFusedRow = kFusedTX + 4, kFusedPlane = kFusedRow * (kFusedTY + 4);
struct FusedArgs {
  const void* uin;
  void* uout;
  const void* src;
  const void* decay;
  const int* tab;
  const void* coef;
  uint32_t ps;
  int pitch, nx, ny, px, py, ntx, nty, nmom, nodd, nd;
  double tau_odd, tau_even;
};
size_t fused_lds_bytes(int storage, int nmom, int nd);
hipError_t launch_fused(int storage, const FusedArgs& f, hipStream_t stream);

// FP64 diagnostics of a state: mass of plane 0 (times cell area is applied on
// the host), sum of squares and max |u| over all valid points, count of
// non-finite values.  part must hold 4 * nblocks doubles, out 4 doubles.
struct DiagArgs {
  const void* u;
  const int* plane_nx;  // valid points per plane along x
  const int* plane_ny;  // valid rows per plane
  int nplanes;
  int64_t plane_stride;
  int pitch;
  int rows_per_block;
  int blocks_per_plane;
  double* part;
  double* out;
};
hipError_t launch_diagnostics(int storage, const DiagArgs& a, hipStream_t stream);
int diag_blocks(int nplanes, int max_rows, int rows_per_block);

}  // namespace starmap
