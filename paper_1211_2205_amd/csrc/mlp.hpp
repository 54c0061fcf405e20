// Launch interface of the learned-closure kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "kernels.hpp"

namespace starmap {

constexpr int CLOSURE_PLANES = 11;   // order-4 and order-5 moments of P_5
constexpr int CLOSURE_FEATURES = 101;  // 99 stencil values + 2 material inputs
constexpr int CLOSURE_IN = 128;       // padded input width
constexpr int CLOSURE_HIDDEN = 128;
constexpr int CLOSURE_OUT = 6;        // order-5 moments
constexpr double CLOSURE_EPS = 1e-20; // added to the stencil norm
// parameters of the FP32 blob: W1 (128 x 128), b1, W2 (128 x 128), b2, W3 (6 x 128), b3
constexpr int CLOSURE_PARAMS = CLOSURE_HIDDEN * CLOSURE_IN + CLOSURE_HIDDEN + CLOSURE_HIDDEN * CLOSURE_HIDDEN +
                               CLOSURE_HIDDEN + CLOSURE_OUT * CLOSURE_HIDDEN + CLOSURE_OUT;

// Network as the fused kernel reads it: bfloat16 weight rows of W1, W2 and W3
// (padded to 16 rows of zeros), then FP32 biases (b3 padded to 16).
struct ClosureNet {
  uint16_t w[(2 * CLOSURE_HIDDEN + 16) * CLOSURE_IN];
  float b1[CLOSURE_HIDDEN];
  float b2[CLOSURE_HIDDEN];
  float b3[16];
};

// One order-6 coupling of an order-5 output: -m * D u_k along axis (0 x, 1 y);
// cell = 1 if plane k is cell-centred along that axis.
struct ClosureTerm {
  int k, axis, cell, pad;
  double m;
};

// Geometry of the closure inputs and outputs in a solver's state.
struct ClosureGeo {
  // input moments: plane, public extents, nodal flags per axis
  int k[CLOSURE_PLANES], pnx[CLOSURE_PLANES], pny[CLOSURE_PLANES], nodex[CLOSURE_PLANES], nodey[CLOSURE_PLANES];
  int nx, ny, px, py, pitch;
  int dk_a, dk_t;  // decay planes: sigma_a on G11, sigma_a + sigma_s on G11
  int64_t plane_stride;
  double dx, dy;
  // outputs: closure plane (inference), public extents, nodal flags
  int q[CLOSURE_OUT], out_nx[CLOSURE_OUT], out_ny[CLOSURE_OUT], out_nodex[CLOSURE_OUT], out_nodey[CLOSURE_OUT];
  // order-6 couplings of each output (training targets)
  int nterm[CLOSURE_OUT];
  ClosureTerm term[CLOSURE_OUT][4];
};

// The odd sweep of a P_5 closure solver fused with the closure network: one
// row per odd moment (orders 1, 3, 5), with its couplings to the even moments
// in the order of the rows of M_x, then M_y, and their coefficients
// -M(k, j) / dx, -M(k, j) / dy.
struct ClosureOddRow {
  int k;        // plane of the moment (orders 1 and 3: updated in place)
  int node_x;   // 1: grid G21 (nodal in x, cell-centred in y); 0: grid G12
  int dk;       // decay plane
  int src;      // source plane (absolute plane index) or -1
  int o;        // order-5 output index 0..5 (read and written through the order-5 buffers), or -1
  int nx, ny;   // couplings along x and y
  int xk[4], xcell[4], yk[4], ycell[4];  // input plane; 1 if the input is cell-centred along the axis
  double xc[4], yc[4];
};
constexpr int CLOSURE_ODD_ROWS = 12;
struct ClosureOdd {
  ClosureOddRow r[CLOSURE_ODD_ROWS];
  double tau;
};

// One instance of a batched run of closure solvers (device table): its state
// planes, the two homes of its order-5 moments (state planes a5, closure
// planes b5), decay planes, sub-step lengths, sweep count, geometry and odd
// rows.
struct ClosureInst {
  void* u;
  void* a5;
  void* b5;
  const void* decay;
  double tau_full, tau_half;
  int nsweeps, pad;
  ClosureGeo G;
  ClosureOdd odd;
};

struct GemmArgs {
  const float* A;
  int64_t sam, sak;
  const float* B;
  int64_t sbk, sbn;
  float* P;   // split partials, splits x M x N
  int M, N, K;
  int kchunk; // K per split, a multiple of 32
};

enum EpiMode : int { EPI_STORE = 0, EPI_GELU = 1, EPI_GELU_GRAD = 2 };

struct EpiArgs {
  const float* P;
  int splits, M, N;
  const float* bias;  // may be null
  int mode;
  const float* aux;   // EPI_GELU_GRAD: pre-activations
  int64_t ldaux;
  float* out;         // EPI_STORE: sum (+ bias); EPI_GELU: pre-activation; EPI_GELU_GRAD: sum * gelu'(aux)
  int64_t ldo;
  float* out2;        // EPI_GELU: gelu(pre-activation)
};

hipError_t launch_gemm(const GemmArgs& g, int splits, const EpiArgs& e, hipStream_t stream);
hipError_t launch_colsum(const float* X, int M, int N, int64_t ld, float* part, float* out, hipStream_t stream);
int colsum_part_floats(int M, int N);
hipError_t launch_mse(const float* Y, const float* T, int64_t count, float* dY, double* part, int nblocks,
                      double* out, hipStream_t stream);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t stream);
hipError_t launch_closure_samples(int storage, const void* U, const void* decay, const ClosureGeo& G,
                                  const int* pts, int count, float* feat, float* targ, float* nu,
                                  hipStream_t stream);
hipError_t launch_closure_infer(int storage, void* U, const void* decay, const ClosureGeo& G, const ClosureNet* net,
                                hipStream_t stream);
// The odd sweep of a P_5 closure solver with the network evaluated in the same
// kernel: reads the order-5 moments from in5 (plane r of output r at
// in5 + r * plane_stride) and writes their updates to out5; updates the
// orders 1 and 3 in place.
hipError_t launch_closure_sweep(int storage, void* U, const void* in5, void* out5, const void* decay,
                                const ClosureGeo& G, const ClosureNet* net, const ClosureOdd& odd,
                                hipStream_t stream);
// Odd sweep j of a batched run of closure solvers (FUSED kernel, BATCH mode):
// the first n_active instances of insts, evaluation blocks numbered from
// bfirst[i]; one network for all.
hipError_t launch_closure_batch(int storage, const ClosureInst* insts, const int* bfirst, int n_active, int blocks,
                                int j, const ClosureNet* net, hipStream_t stream);
// The network alone over a batch of closure solvers (BATCH mode without the
// fused sweep): every running instance's closure planes, which its odd sweep
// then reads as sources.
hipError_t launch_closure_batch_net(int storage, const ClosureInst* insts, const int* bfirst, int n_active, int blocks,
                                    const ClosureNet* net, hipStream_t stream);
size_t closure_infer_lds_bytes();

}  // namespace starmap
