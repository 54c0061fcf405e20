// Learned closure of the P_5 hierarchy on gfx950: the network's training
// kernels (BF16 MFMA matrix products with FP32 accumulation, GELU, loss,
// Adam), the extraction of training samples from a high-order state, and the
// fused closure kernel that evaluates the network at every point of a P_5
// state before an odd sweep.
//
// The closure replaces the order-6 flux the P_N truncation drops (the moment
// system is closed by zeroing order N + 1, Sect. 2) with a network of the
// local order-4/5 data:
//   inputs  : 3 x 3 array stencils of the eleven order-4/5 moments divided by
//             their norm nu, log10(sigma_a + 0.01), log10(sigma_s + 0.01),
//             zero padding to 128;
//   network : 128 -> 128 -> 128 -> 6, GELU after the hidden layers;
//   output  : g = nu * y / dx added to the residual of the six order-5 moments.
// Matrix-product operands are rounded to bfloat16 (nearest, ties to even);
// accumulation, biases and activations before rounding are FP32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "mlp.hpp"

namespace starmap {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ scalar helpers
__device__ __forceinline__ uint32_t bf16_bits(float v) { return from_c<bf16>(v).bits; }

// Correctly rounded double -> bfloat16: round to odd into FP32 (24 bits, at
// least two more than bfloat16 keeps), then to nearest even.
__device__ __forceinline__ uint32_t bf16_bits(double v) {
  float f = __double2float_rz(v);
  if (double(f) != v) f = __uint_as_float(__float_as_uint(f) | 1u);
  return bf16_bits(f);
}

__device__ __forceinline__ float bf16_value(uint32_t bits) { return __uint_as_float(bits << 16); }

// The same rounding (nearest, ties to even) by the conversion instruction.
__device__ __forceinline__ uint32_t bf16_hw(float v) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
}
__device__ __forceinline__ uint32_t bf16_in(float v) { return bf16_hw(v); }
__device__ __forceinline__ uint32_t bf16_in(double v) { return bf16_bits(v); }

// GELU z Phi(z), Phi the standard normal distribution function, with erf
// from Abramowitz & Stegun, Handbook of Mathematical Functions, formula 7.1.26
// (|error| <= 1.5e-7 on the real line).  Training and inference use this one
// definition.
__device__ __forceinline__ float normal_cdf(float z) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
  const float poly =
      t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f), 0.254829592f);
  const float erf_abs = 1.0f - poly * __expf(-x * x);
  return 0.5f * (1.0f + copysignf(erf_abs, z));
}
__device__ __forceinline__ float gelu(float z) { return z * normal_cdf(z); }
// d/dz z Phi(z) = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad(float z) {
  return normal_cdf(z) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ f32x4 mfma16(uint4 a, uint4 b, f32x4 c) {
  // D[i][j] += sum_k A[i][k] B[k][j], 16 x 16 x 32: lane l holds A[l % 16][8 (l / 16) + e]
  // and B[8 (l / 16) + e][l % 16] (e = 0..7), and D[4 (l / 16) + r][l % 16] (r = 0..3)
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                  0, 0, 0);
}

__device__ __forceinline__ uint4 pack8(const uint32_t (&h)[8]) {
  return make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
}

// ------------------------------------------------------------ training GEMM
// P[z][m][n] = sum over k in split z of bf16(A(m, k)) * bf16(B(k, n)), with
// A(m, k) = A[m sam + k sak] and B(k, n) = B[k sbk + n sbn].  64 x 64 outputs
// per workgroup; four waves of 32 x 32; K in steps of 32 through LDS.
constexpr int GT = 64;        // output tile edge
constexpr int GK = 32;        // K step
constexpr int GLD = GK + 8;   // LDS row of one tile row / column (bf16), padded

__global__ void __launch_bounds__(256) gemm_bf16_kernel(const GemmArgs g) {
  __shared__ __align__(16) uint16_t As[GT * GLD];
  __shared__ __align__(16) uint16_t Bs[GT * GLD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
  const int kb = blockIdx.z * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging: thread t fills row (or column) t / 4, k offsets 8 (t % 4) .. + 7
  const int sr = tid >> 2, sk = (tid & 3) * 8;
  for (int k0 = kb; k0 < ke; k0 += GK) {
    uint32_t ha[8], hb[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + sk + e;
      const int m = m0 + sr, n = n0 + sr;
      const float av = (m < g.M && k < ke) ? g.A[int64_t(m) * g.sam + int64_t(k) * g.sak] : 0.f;
      const float bv = (n < g.N && k < ke) ? g.B[int64_t(k) * g.sbk + int64_t(n) * g.sbn] : 0.f;
      ha[e] = bf16_bits(av);
      hb[e] = bf16_bits(bv);
    }
    __syncthreads();  // the previous step's fragments are read
    *reinterpret_cast<uint4*>(&As[sr * GLD + sk]) = pack8(ha);
    *reinterpret_cast<uint4*>(&Bs[sr * GLD + sk]) = pack8(hb);
    __syncthreads();
    const int fk = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint4 a = *reinterpret_cast<const uint4*>(&As[(wm + 16 * i + (lane & 15)) * GLD + fk]);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const uint4 b = *reinterpret_cast<const uint4*>(&Bs[(wn + 16 * j + (lane & 15)) * GLD + fk]);
        acc[i][j] = mfma16(a, b, acc[i][j]);
      }
    }
  }
  float* P = g.P + int64_t(blockIdx.z) * g.M * g.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m < g.M && n < g.N) P[int64_t(m) * g.N + n] = acc[i][j][r];
      }
}

// Sum of the split partials in split order, then the epilogue.
__global__ void __launch_bounds__(256) gemm_epilogue_kernel(const EpiArgs e) {
  const int64_t total = int64_t(e.M) * e.N;
  for (int64_t t = blockIdx.x * int64_t(256) + threadIdx.x; t < total; t += int64_t(gridDim.x) * 256) {
    const int m = int(t / e.N), n = int(t % e.N);
    float acc = 0.f;
    for (int z = 0; z < e.splits; ++z) acc += e.P[z * total + t];
    if (e.bias) acc += e.bias[n];
    if (e.mode == EPI_STORE) {
      e.out[int64_t(m) * e.ldo + n] = acc;
    } else if (e.mode == EPI_GELU) {
      e.out[int64_t(m) * e.ldo + n] = acc;
      e.out2[int64_t(m) * e.ldo + n] = gelu(acc);
    } else {  // EPI_GELU_GRAD
      e.out[int64_t(m) * e.ldo + n] = acc * gelu_grad(e.aux[int64_t(m) * e.ldaux + n]);
    }
  }
}

// Column sums of X (M x N, row stride ld) in a fixed order: partial sums of
// row chunks, then the chunks in order.
constexpr int CS_ROWS = 256;
__global__ void __launch_bounds__(256) colsum_partial_kernel(const float* X, int M, int N, int64_t ld, float* part) {
  __shared__ float s[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
  const int r0 = blockIdx.y * CS_ROWS, r1 = min(M, r0 + CS_ROWS);
  float a = 0.f;
  if (c < N)
    for (int r = r0 + ph; r < r1; r += 4) a += X[int64_t(r) * ld + c];
  s[ph][threadIdx.x & 63] = a;
  __syncthreads();
  if (ph == 0 && c < N) part[int64_t(blockIdx.y) * N + c] = ((s[0][threadIdx.x] + s[1][threadIdx.x]) + s[2][threadIdx.x]) + s[3][threadIdx.x];
}

__global__ void __launch_bounds__(256) colsum_final_kernel(const float* part, int chunks, int N, float* out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= N) return;
  float a = 0.f;
  for (int z = 0; z < chunks; ++z) a += part[int64_t(z) * N + c];
  out[c] = a;
}

// dY = 2 (Y - T) / count and per-block partial sums of (Y - T)^2 in FP64.
__global__ void __launch_bounds__(256) mse_kernel(const float* Y, const float* T, int64_t count, float* dY,
                                                  double* part) {
  __shared__ double s[256];
  double a = 0.0;
  const float scale = 2.0f / float(count);
  for (int64_t t = blockIdx.x * int64_t(256) + threadIdx.x; t < count; t += int64_t(gridDim.x) * 256) {
    const float d = Y[t] - T[t];
    dY[t] = scale * d;
    a += double(d) * double(d);
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(256) sum_final_kernel(const double* part, int n, double scale, double* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = s[0] * scale;
}

// Adam with bias correction; c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void __launch_bounds__(256) adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * int64_t(256) + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// ------------------------------------------------------------ closure inputs
// Public index a of a moment's array along an axis -> internal storage index
// (nodes of a periodic axis are stored modulo n).
__device__ __forceinline__ int internal_index(int a, int node, int periodic, int n) {
  return (node && periodic) ? (a + 1) % n : a;
}

// The 99 stencil values at evaluation point (i, j) (moment, then b, then a)
// and the two material inputs.
template <typename T, typename C>
__device__ __forceinline__ void stencil_value(const T* __restrict__ U, const ClosureGeo& G, int p, int i, int j,
                                              int a, int b, C* out) {
  const int ii = min(max(i + a, 0), G.pnx[p] - 1);
  const int jj = min(max(j + b, 0), G.pny[p] - 1);
  const int X = internal_index(ii, G.nodex[p], G.px, G.nx);
  const int Y = internal_index(jj, G.nodey[p], G.py, G.ny);
  *out = to_c(U[int64_t(G.k[p]) * G.plane_stride + int64_t(Y) * G.pitch + X]);
}

template <typename C>
__device__ __forceinline__ void sigma_inputs(const C* __restrict__ decay, const ClosureGeo& G, int i, int j, C* fa,
                                             C* fs) {
  const int ci = min(i, G.nx - 1), cj = min(j, G.ny - 1);
  const int64_t o = int64_t(cj) * G.pitch + ci;
  const C sa = decay[int64_t(G.dk_a) * G.plane_stride + o];
  const C st = decay[int64_t(G.dk_t) * G.plane_stride + o];
  *fa = log10(sa + C(0.01));
  *fs = log10((st - sa) + C(0.01));
}

// Training samples from a state of order >= 6: inputs (count x 128, FP32) and
// targets F_k dx / nu (count x 6) at cells (i, j), one thread per sample.
// targ may be null (inputs only); nu_out, if not null, receives nu per sample.
template <typename T>
__global__ void __launch_bounds__(256) closure_samples_kernel(const T* __restrict__ U,
                                                              const typename ComputeOf<T>::type* __restrict__ decay,
                                                              const ClosureGeo G, const int* __restrict__ pts,
                                                              int count, float* __restrict__ feat,
                                                              float* __restrict__ targ, float* __restrict__ nu_out) {
  using C = typename ComputeOf<T>::type;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= count) return;
  const int i = pts[2 * s], j = pts[2 * s + 1];
  C ss = C(0);
  for (int p = 0; p < CLOSURE_PLANES; ++p)
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a) {
        C v;
        stencil_value(U, G, p, i, j, a, b, &v);
        ss += v * v;
      }
  const C nu = sqrt(ss) + C(CLOSURE_EPS);
  float* f = feat + int64_t(s) * CLOSURE_IN;
  int q = 0;
  for (int p = 0; p < CLOSURE_PLANES; ++p)
    for (int b = -1; b <= 1; ++b)
      for (int a = -1; a <= 1; ++a) {
        C v;
        stencil_value(U, G, p, i, j, a, b, &v);
        f[q++] = float(v / nu);
      }
  C fa, fs;
  sigma_inputs(decay, G, i, j, &fa, &fs);
  f[q++] = float(fa);
  f[q++] = float(fs);
  for (; q < CLOSURE_IN; ++q) f[q] = 0.f;
  if (nu_out) nu_out[s] = float(nu);
  if (!targ) return;
  // targets: the order-6 part of the odd residual at the order-5 points
  for (int o = 0; o < CLOSURE_OUT; ++o) {
    const int X = internal_index(i, G.out_nodex[o], G.px, G.nx);
    const int Y = internal_index(j, G.out_nodey[o], G.py, G.ny);
    C F = C(0);
    for (int t = 0; t < G.nterm[o]; ++t) {
      const ClosureTerm& ct = G.term[o][t];
      const T* up = U + int64_t(ct.k) * G.plane_stride;
      C d;
      if (ct.axis == 0) {  // x difference; the input shares the output's y index
        const int lo = ct.cell ? map_axis(X - 1, G.nx, G.px, 1) : map_axis(X, G.nx, G.px, 0);
        const int hi = ct.cell ? map_axis(X, G.nx, G.px, 1) : map_axis(X + 1, G.nx, G.px, 0);
        d = (to_c(up[int64_t(Y) * G.pitch + hi]) - to_c(up[int64_t(Y) * G.pitch + lo])) / C(G.dx);
      } else {
        const int lo = ct.cell ? map_axis(Y - 1, G.ny, G.py, 1) : map_axis(Y, G.ny, G.py, 0);
        const int hi = ct.cell ? map_axis(Y, G.ny, G.py, 1) : map_axis(Y + 1, G.ny, G.py, 0);
        d = (to_c(up[int64_t(hi) * G.pitch + X]) - to_c(up[int64_t(lo) * G.pitch + X])) / C(G.dy);
      }
      F -= C(ct.m) * d;
    }
    targ[int64_t(s) * CLOSURE_OUT + o] = float(F * C(G.dx) / nu);
  }
}

// ------------------------------------------------------------ fused closure
// Every workgroup keeps the network and loops over blocks of 64 evaluation
// points of the (nx + 1) x (ny + 1) index domain: gather and normalise the
// inputs, three MFMA layers, then nu * y / dx into the closure planes of the
// order-5 moments.  The layers are computed transposed, H^T = W X^T: the
// weights are the A operand and stay in registers (wave w owns hidden units
// [32 w, 32 w + 32)), the activations are the B operand, read from LDS as
// [point][unit] rows, and each lane's four outputs (consecutive units of one
// point) go back with one 8-byte LDS write.
constexpr int CB = 64;               // evaluation points per block
constexpr int LDW = CLOSURE_IN + 8;  // LDS row of one point's activations (bf16), padded

// The odd update of one odd moment of P_5 at the internal point (X, Y) of its
// grid, with the couplings in the order of the sweep kernel (x terms, then y
// terms), the source, then the closure term g: u + tau (W - c u) E(-c tau).
template <typename T, typename C>
__device__ __forceinline__ C closure_odd_update(const T* __restrict__ U, const ClosureOddRow& r, const ClosureGeo& G,
                                                int X, int Y, C u, C g, C c, C E, C tau) {
  // plane bases are wave-uniform; the lane's offsets are 32-bit byte offsets
  // within a plane (planes stay below 2^31 bytes), so every load takes a
  // scalar base and one offset register
  const uint64_t ps = uint64_t(G.plane_stride);
  constexpr uint32_t TS = sizeof(T);
  const char* base = reinterpret_cast<const char*>(U);
  auto val = [&](int k, uint32_t off) {
    return to_c(*reinterpret_cast<const T*>(base + uint64_t(uint32_t(k)) * ps * TS + off));
  };
  const uint32_t row = uint32_t(Y) * uint32_t(G.pitch);
  C W = C(0);
  for (int t = 0; t < r.nx; ++t) {
    const int lo = r.xcell[t] ? map_axis(X - 1, G.nx, G.px, 1) : map_axis(X, G.nx, G.px, 0);
    const int hi = r.xcell[t] ? map_axis(X, G.nx, G.px, 1) : map_axis(X + 1, G.nx, G.px, 0);
    W = couple(W, C(r.xc[t]), val(r.xk[t], (row + uint32_t(hi)) * TS), val(r.xk[t], (row + uint32_t(lo)) * TS));
  }
  for (int t = 0; t < r.ny; ++t) {
    const int lo = r.ycell[t] ? map_axis(Y - 1, G.ny, G.py, 1) : map_axis(Y, G.ny, G.py, 0);
    const int hi = r.ycell[t] ? map_axis(Y, G.ny, G.py, 1) : map_axis(Y + 1, G.ny, G.py, 0);
    W = couple(W, C(r.yc[t]), val(r.yk[t], (uint32_t(hi) * uint32_t(G.pitch) + uint32_t(X)) * TS),
               val(r.yk[t], (uint32_t(lo) * uint32_t(G.pitch) + uint32_t(X)) * TS));
  }
  if (r.src >= 0) W += val(r.src, (row + uint32_t(X)) * TS);
  if (r.o >= 0) W += g;
  return sub_step(u, W, c, E, tau);
}

// FUSED = false: the closure terms g = nu y / dx of every evaluation point go
// to the closure planes, which the odd sweep then reads like source planes.
// FUSED = true: the same network, then the odd sweep of P_5 at the block's
// points in the same workgroup (every odd moment at every evaluation point
// that lies on its grid), the order-5 moments read from in5 and written to
// out5 (out of place, so every workgroup's stencils see the state of the
// start of the sweep), orders 1 and 3 in place (nothing else reads them).
//
// BATCH = true: odd sweep number j of a batched run of closure solvers
// sharing one network; instance i (of the n_active still running, sorted by
// their sweep counts) owns the evaluation blocks [bfirst[i], bfirst[i + 1])
// and brings its own state, geometry and odd rows (insts[i]); the arguments
// U .. odd are unused.  With FUSED the kernel performs the odd sweeps as
// above; without, it writes every instance's closure planes, and a batched
// odd sweep follows.
template <typename T, bool FUSED, bool BATCH>
__global__ void __launch_bounds__(256, 3) closure_infer_kernel(T* __restrict__ U0, const T* __restrict__ in5_0,
                                                            T* __restrict__ out5_0,
                                                            const typename ComputeOf<T>::type* __restrict__ decay0,
                                                            const ClosureGeo G0, const ClosureNet* __restrict__ net,
                                                            const ClosureOdd odd0,
                                                            const ClosureInst* __restrict__ insts,
                                                            const int* __restrict__ bfirst, const int n_active,
                                                            const int jsweep) {
  using C = typename ComputeOf<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* Xa = reinterpret_cast<uint16_t*>(smem);  // [64][LDW] inputs, then layer-2 activations
  uint16_t* Xb = Xa + CB * LDW;                      // [64][LDW] layer-1 activations
  uint16_t* W3 = Xb + CB * LDW;                      // [16][LDW] output layer, rows >= 6 zero
  C* nu_s = reinterpret_cast<C*>(W3 + 16 * LDW);     // [64]
  C* part = nu_s + CB;                                    // [4][64] partial sums of squares per wave
  int* otab = reinterpret_cast<int*>(part + 4 * CB);  // [5][8] output plane, extents, nodal flags
  C* gsh = reinterpret_cast<C*>(otab + 5 * 8);        // FUSED: [6][64] closure terms of the block
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int fk = 8 * (lane >> 4);

  // the output geometry, indexed per lane below, from LDS (indexing the
  // kernel argument per lane would turn every access into a dependent load);
  // batched: each block's instance's, written at the start of the block
  auto fill_otab = [&](const ClosureGeo& G) {
    if (tid < 5 * 8) {
      const int f = tid >> 3, o = tid & 7;
      int v = 0;
      if (o < CLOSURE_OUT)
        v = f == 0 ? G.q[o] : f == 1 ? G.out_nx[o] : f == 2 ? G.out_ny[o] : f == 3 ? G.out_nodex[o] : G.out_nodey[o];
      otab[tid] = v;
    }
  };
  if constexpr (!FUSED && !BATCH) fill_otab(G0);

  // this wave's weight fragments: rows 32 w + 16 mi + (lane % 16), k = 32 ks + fk
  const uint4* wv = reinterpret_cast<const uint4*>(net->w);  // rows of CLOSURE_IN / 8 uint4
  uint4 wf[2][2][4];
#pragma unroll
  for (int layer = 0; layer < 2; ++layer)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int row = layer * CLOSURE_HIDDEN + 32 * w + 16 * mi + (lane & 15);
        wf[layer][mi][ks] = wv[row * (CLOSURE_IN / 8) + (32 * ks + fk) / 8];
      }
  for (int e = tid; e < 16 * (CLOSURE_IN / 8); e += 256)
    *reinterpret_cast<uint4*>(&W3[(e / (CLOSURE_IN / 8)) * LDW + (e % (CLOSURE_IN / 8)) * 8]) =
        wv[2 * CLOSURE_HIDDEN * (CLOSURE_IN / 8) + e];
  float b3[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) b3[r] = net->b3[4 * (lane >> 4) + r];

  const int nblk = BATCH ? bfirst[n_active] : ((G0.nx + 1) * (G0.ny + 1) + CB - 1) / CB;
  for (int gblk = blockIdx.x; gblk < nblk; gblk += gridDim.x) {
    // this block's instance (batched runs) and its data
    int inst = 0;
    if constexpr (BATCH) {
      int lo = 0, hi = n_active - 1;  // last instance with bfirst[i] <= gblk
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bfirst[mid] <= gblk) lo = mid; else hi = mid - 1;
      }
      inst = lo;
    }
    const int blk = BATCH ? gblk - bfirst[inst] : gblk;
    const ClosureGeo& G = BATCH ? insts[inst].G : G0;
    const ClosureOdd& odd = BATCH ? insts[inst].odd : odd0;
    T* const U = BATCH ? static_cast<T*>(insts[inst].u) : U0;
    const C* const decay = BATCH ? static_cast<const C*>(insts[inst].decay) : decay0;
    // fused: the order-5 moments move between the state planes and the
    // closure planes at every odd sweep, and odd sweep j of a batched run
    // reads them where j / 2 earlier odd sweeps left them (the network alone
    // reads them in the state planes)
    const bool flip = BATCH && FUSED && ((jsweep >> 1) & 1);
    const T* const in5 = BATCH ? static_cast<const T*>(flip ? insts[inst].b5 : insts[inst].a5) : in5_0;
    T* const out5 = BATCH ? static_cast<T*>(flip ? insts[inst].a5 : insts[inst].b5) : out5_0;
    const C tau = BATCH ? C((jsweep == 0 || jsweep == insts[inst].nsweeps - 1) ? insts[inst].tau_half
                                                                             : insts[inst].tau_full)
                        : C(odd0.tau);
    const int NXE = G.nx + 1, total = NXE * (G.ny + 1);
    // 1. inputs: wave w gathers moments w, w + 4, w + 8 of point lane
    const int pt = blk * CB + lane;
    const bool live = pt < total;
    const int i = live ? pt % NXE : 0, j = live ? pt / NXE : 0;
    // clamped (or wrapped) columns and rows of the stencil, per axis class:
    // [0] cell-centred, [1] nodal
    int colx[2][3], rowy[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      colx[0][a] = min(max(i + a - 1, 0), G.nx - 1);
      const int xn = min(max(i + a - 1, 0), G.nx - G.px);
      colx[1][a] = G.px ? (xn + 1 == G.nx ? 0 : xn + 1) : xn;
      rowy[0][a] = min(max(j + a - 1, 0), G.ny - 1) * G.pitch;
      const int yn = min(max(j + a - 1, 0), G.ny - G.py);
      rowy[1][a] = (G.py ? (yn + 1 == G.ny ? 0 : yn + 1) : yn) * G.pitch;
    }
    // the material inputs of this point (wave 3), loaded now so that they
    // arrive with the stencil
    C sig_a = C(0), sig_t = C(0);
    if (w == 3) {
      const int64_t o = int64_t(min(j, G.ny - 1)) * G.pitch + min(i, G.nx - 1);
      sig_a = decay[int64_t(G.dk_a) * G.plane_stride + o];
      sig_t = decay[int64_t(G.dk_t) * G.plane_stride + o];
    }
    // two passes over the stencil (the second re-reads cached values): the
    // sum of squares, then the normalised inputs
    C ss = C(0);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int p = w + 4 * t;
      if (p < CLOSURE_PLANES) {
        const T* up = p < 5 ? U + int64_t(G.k[p]) * G.plane_stride : in5 + int64_t(p - 5) * G.plane_stride;
        const int cx = G.nodex[p], cy = G.nodey[p];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          const C v = to_c(up[rowy[cy][q / 3] + colx[cx][q % 3]]);
          ss += v * v;
        }
      }
    }
    // the second pass's first plane (every wave has one) is re-read while the
    // norm is reduced across the waves
    C v0[9];
    {
      const T* up = U + int64_t(G.k[w]) * G.plane_stride;  // w < 4: an order-4 plane
      const int cx = G.nodex[w], cy = G.nodey[w];
#pragma unroll
      for (int q = 0; q < 9; ++q) v0[q] = to_c(up[rowy[cy][q / 3] + colx[cx][q % 3]]);
    }
    __syncthreads();  // the previous block's reads of Xa, nu_s, part and otab are done
    part[w * CB + lane] = ss;
    if constexpr (!FUSED && BATCH) fill_otab(G);
    __syncthreads();
    const C nu = sqrt(((part[lane] + part[CB + lane]) + part[2 * CB + lane]) + part[3 * CB + lane]) + C(CLOSURE_EPS);
    const C rnu = C(1) / nu;
#pragma unroll
    for (int q = 0; q < 9; ++q) Xa[lane * LDW + 9 * w + q] = uint16_t(bf16_in(v0[q] * rnu));
#pragma unroll
    for (int t = 1; t < 3; ++t) {
      const int p = w + 4 * t;
      if (p < CLOSURE_PLANES) {
        const T* up = p < 5 ? U + int64_t(G.k[p]) * G.plane_stride : in5 + int64_t(p - 5) * G.plane_stride;
        const int cx = G.nodex[p], cy = G.nodey[p];
        // all nine loads first, so they are in flight together
        C v[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q] = to_c(up[rowy[cy][q / 3] + colx[cx][q % 3]]);
#pragma unroll
        for (int q = 0; q < 9; ++q) Xa[lane * LDW + 9 * p + q] = uint16_t(bf16_in(v[q] * rnu));
      }
    }
    if (w == 3) {
      const C fa = log10(sig_a + C(0.01)), fs = log10((sig_t - sig_a) + C(0.01));
      Xa[lane * LDW + 99] = uint16_t(bf16_bits(fa));
      Xa[lane * LDW + 100] = uint16_t(bf16_bits(fs));
      for (int q = 101; q < CLOSURE_IN; ++q) Xa[lane * LDW + q] = 0;
      nu_s[lane] = nu;
    }
    __syncthreads();

    // 2. hidden layers: H^T (units x points) = W X^T; wave w: 32 units x 64 points
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      const uint16_t* Xin = layer == 0 ? Xa : Xb;
      uint16_t* Xout = layer == 0 ? Xb : Xa;
      f32x4 acc[2][4];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 4; ++nj) acc[mi][nj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
        for (int nj = 0; nj < 4; ++nj) {
          const uint4 xf = *reinterpret_cast<const uint4*>(&Xin[(16 * nj + (lane & 15)) * LDW + 32 * ks + fk]);
#pragma unroll
          for (int mi = 0; mi < 2; ++mi) acc[mi][nj] = mfma16(wf[layer][mi][ks], xf, acc[mi][nj]);
        }
      }
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 4; ++nj) {
          // rows: units 32 w + 16 mi + 4 (lane / 16) + r; column: point 16 nj + lane % 16
          const float4 bv = *reinterpret_cast<const float4*>((layer == 0 ? net->b1 : net->b2) + 32 * w + 16 * mi +
                                                             4 * (lane >> 4));
          uint32_t h[4];
          h[0] = bf16_hw(gelu(acc[mi][nj][0] + bv.x));
          h[1] = bf16_hw(gelu(acc[mi][nj][1] + bv.y));
          h[2] = bf16_hw(gelu(acc[mi][nj][2] + bv.z));
          h[3] = bf16_hw(gelu(acc[mi][nj][3] + bv.w));
          const int m = 16 * nj + (lane & 15);
          const int n = 32 * w + 16 * mi + 4 * (lane >> 4);
          *reinterpret_cast<uint2*>(&Xout[m * LDW + n]) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
        }
      __syncthreads();
    }

    // 3. output layer: Y^T (16 x points) = W3 X^T; wave w takes points [16 w, 16 w + 16)
    f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const uint4 af = *reinterpret_cast<const uint4*>(&W3[(lane & 15) * LDW + 32 * ks + fk]);
      const uint4 xf = *reinterpret_cast<const uint4*>(&Xa[(16 * w + (lane & 15)) * LDW + 32 * ks + fk]);
      y = mfma16(af, xf, y);
    }
    const int m = 16 * w + (lane & 15);  // point of this lane
    const int p2 = blk * CB + m;
    if (!FUSED) {
      if (p2 < total) {
        const int pi = p2 % NXE, pj = p2 / NXE;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int o = 4 * (lane >> 4) + r;  // output of this lane
          if (o >= CLOSURE_OUT || pi >= otab[8 + o] || pj >= otab[16 + o]) continue;
          const int X = internal_index(pi, otab[24 + o], G.px, G.nx);
          const int Y = internal_index(pj, otab[32 + o], G.py, G.ny);
          const C g = nu_s[m] * C(y[r] + b3[r]) / C(G.dx);
          U[int64_t(otab[o]) * G.plane_stride + int64_t(Y) * G.pitch + X] = from_c<T>(g);
        }
      }
      continue;
    }
    // 4. (fused) the closure terms of the block into LDS, then the odd update:
    // wave w takes odd rows w, w + 4, w + 8, lane = point of the block
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * (lane >> 4) + r;
      if (o < CLOSURE_OUT) gsh[o * CB + m] = nu_s[m] * C(y[r] + b3[r]) / C(G.dx);
    }
    __syncthreads();
    if (pt < total) {  // the point of this lane: (i, j) of the gather above
      // decay and E(-c tau) per output grid, reloaded when a row's decay plane differs
      int dk21 = -1, dk12 = -1;
      C c21 = C(0), e21 = C(0), c12 = C(0), e12 = C(0);
      const int w0 = __builtin_amdgcn_readfirstlane(w);
      for (int q = w0; q < CLOSURE_ODD_ROWS; q += 4) {
        const ClosureOddRow& r = odd.r[q];
        const int nd = r.node_x;
        // the row's grid: G21 has nx + 1 - px by ny points, G12 nx by ny + 1 - py
        if (nd ? (i >= G.nx + 1 - G.px || j >= G.ny) : (i >= G.nx || j >= G.ny + 1 - G.py)) continue;
        const int X = nd ? internal_index(i, 1, G.px, G.nx) : i;
        const int Y = nd ? j : internal_index(j, 1, G.py, G.ny);
        const int64_t off = int64_t(Y) * G.pitch + X;
        if (nd && r.dk != dk21) {
          c21 = decay[int64_t(r.dk) * G.plane_stride + off];
          e21 = expm1div(-c21 * tau);
          dk21 = r.dk;
        } else if (!nd && r.dk != dk12) {
          c12 = decay[int64_t(r.dk) * G.plane_stride + off];
          e12 = expm1div(-c12 * tau);
          dk12 = r.dk;
        }
        const T* src = r.o >= 0 ? in5 + int64_t(r.o) * G.plane_stride : U + int64_t(r.k) * G.plane_stride;
        const C u = to_c(src[off]);
        const C g = r.o >= 0 ? gsh[r.o * CB + lane] : C(0);
        const C v = closure_odd_update(U, r, G, X, Y, u, g, nd ? c21 : c12, nd ? e21 : e12, tau);
        T* dst = r.o >= 0 ? out5 + int64_t(r.o) * G.plane_stride : U + int64_t(r.k) * G.plane_stride;
        dst[off] = from_c<T>(v);
      }
    }
  }
}

// ------------------------------------------------------------ launches
hipError_t launch_gemm(const GemmArgs& g, int splits, const EpiArgs& e, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0 || g.K < 0 || splits < 1) return hipErrorInvalidValue;
  dim3 grid((g.N + GT - 1) / GT, (g.M + GT - 1) / GT, splits);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, stream, g);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  const int64_t total = int64_t(g.M) * g.N;
  const int blocks = int(std::min<int64_t>((total + 255) / 256, 4096));
  hipLaunchKernelGGL(gemm_epilogue_kernel, dim3(blocks), dim3(256), 0, stream, e);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* X, int M, int N, int64_t ld, float* part, float* out, hipStream_t stream) {
  const int chunks = (M + CS_ROWS - 1) / CS_ROWS;
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((N + 63) / 64, chunks), dim3(256), 0, stream, X, M, N, ld, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0, stream, part, chunks, N, out);
  return hipGetLastError();
}

int colsum_part_floats(int M, int N) { return ((M + CS_ROWS - 1) / CS_ROWS) * N; }

hipError_t launch_mse(const float* Y, const float* T, int64_t count, float* dY, double* part, int nblocks,
                      double* out, hipStream_t stream) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, stream, Y, T, count, dY, part);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(sum_final_kernel, dim3(1), dim3(256), 0, stream, part, nblocks, 1.0 / double(count), out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t stream) {
  const int blocks = int(std::min<int64_t>((n + 255) / 256, 1024));
  hipLaunchKernelGGL(adam_kernel, dim3(blocks), dim3(256), 0, stream, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_closure_samples(int storage, const void* U, const void* decay, const ClosureGeo& G,
                                  const int* pts, int count, float* feat, float* targ, float* nu, hipStream_t stream) {
  const dim3 grid((count + 255) / 256);
  switch (storage) {
    case STORE_FP64:
      hipLaunchKernelGGL(closure_samples_kernel<double>, grid, dim3(256), 0, stream,
                         static_cast<const double*>(U), static_cast<const double*>(decay), G, pts, count, feat, targ, nu);
      break;
    case STORE_FP32:
      hipLaunchKernelGGL(closure_samples_kernel<float>, grid, dim3(256), 0, stream,
                         static_cast<const float*>(U), static_cast<const float*>(decay), G, pts, count, feat, targ, nu);
      break;
    case STORE_BF16:
      hipLaunchKernelGGL(closure_samples_kernel<bf16>, grid, dim3(256), 0, stream,
                         static_cast<const bf16*>(U), static_cast<const float*>(decay), G, pts, count, feat, targ, nu);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t closure_infer_lds_bytes() {
  return size_t(2 * CB + 16) * LDW * 2 + size_t(5 * CB) * 8 + 5 * 8 * sizeof(int) + size_t(CLOSURE_OUT * CB) * 8;
}

namespace {
template <typename T, bool FUSED, bool BATCH>
hipError_t launch_infer_t(void* U, const void* in5, void* out5, const void* decay, const ClosureGeo& G,
                          const ClosureNet* net, const ClosureOdd& odd, const ClosureInst* insts, const int* bfirst,
                          int n_active, int j, int blocks, hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  static bool attr = false;
  const size_t lds = closure_infer_lds_bytes();
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&closure_infer_kernel<T, FUSED, BATCH>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((closure_infer_kernel<T, FUSED, BATCH>), dim3(blocks), dim3(256), lds, stream,
                     static_cast<T*>(U), static_cast<const T*>(in5), static_cast<T*>(out5),
                     static_cast<const C*>(decay), G, net, odd, insts, bfirst, n_active, j);
  return hipGetLastError();
}

int device_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
  }
  return cus;
}

// a few workgroups per compute unit, each looping over blocks of points with
// the weights loaded once
int infer_blocks(const ClosureGeo& G) {
  const int total = (G.nx + 1) * (G.ny + 1);
  const int nblk = (total + CB - 1) / CB;
  return std::min(nblk, 3 * device_cus());
}
}  // namespace

hipError_t launch_closure_infer(int storage, void* U, const void* decay, const ClosureGeo& G, const ClosureNet* net,
                                hipStream_t stream) {
  const int blocks = infer_blocks(G);
  ClosureOdd none{};
  // the order-5 inputs sit in U (moments G.k[5 ..], consecutive)
  switch (storage) {
    case STORE_FP64: {
      double* u = static_cast<double*>(U);
      return launch_infer_t<double, false, false>(U, u + int64_t(G.k[5]) * G.plane_stride, nullptr, decay, G, net,
                                                  none, nullptr, nullptr, 0, 0, blocks, stream);
    }
    case STORE_FP32: {
      float* u = static_cast<float*>(U);
      return launch_infer_t<float, false, false>(U, u + int64_t(G.k[5]) * G.plane_stride, nullptr, decay, G, net,
                                                 none, nullptr, nullptr, 0, 0, blocks, stream);
    }
    case STORE_BF16: {
      bf16* u = static_cast<bf16*>(U);
      return launch_infer_t<bf16, false, false>(U, u + int64_t(G.k[5]) * G.plane_stride, nullptr, decay, G, net,
                                                none, nullptr, nullptr, 0, 0, blocks, stream);
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_closure_sweep(int storage, void* U, const void* in5, void* out5, const void* decay,
                                const ClosureGeo& G, const ClosureNet* net, const ClosureOdd& odd,
                                hipStream_t stream) {
  const int blocks = infer_blocks(G);
  switch (storage) {
    case STORE_FP64:
      return launch_infer_t<double, true, false>(U, in5, out5, decay, G, net, odd, nullptr, nullptr, 0, 0, blocks,
                                                 stream);
    case STORE_FP32:
      return launch_infer_t<float, true, false>(U, in5, out5, decay, G, net, odd, nullptr, nullptr, 0, 0, blocks,
                                                stream);
    case STORE_BF16:
      return launch_infer_t<bf16, true, false>(U, in5, out5, decay, G, net, odd, nullptr, nullptr, 0, 0, blocks,
                                               stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_closure_batch_net(int storage, const ClosureInst* insts, const int* bfirst, int n_active, int blocks,
                                    const ClosureNet* net, hipStream_t stream) {
  if (n_active < 1 || blocks < 1) return hipErrorInvalidValue;
  const int grid = std::min(blocks, 3 * device_cus());
  const ClosureGeo G{};
  const ClosureOdd odd{};
  switch (storage) {
    case STORE_FP64:
      return launch_infer_t<double, false, true>(nullptr, nullptr, nullptr, nullptr, G, net, odd, insts, bfirst,
                                                 n_active, 0, grid, stream);
    case STORE_FP32:
      return launch_infer_t<float, false, true>(nullptr, nullptr, nullptr, nullptr, G, net, odd, insts, bfirst,
                                                n_active, 0, grid, stream);
    case STORE_BF16:
      return launch_infer_t<bf16, false, true>(nullptr, nullptr, nullptr, nullptr, G, net, odd, insts, bfirst,
                                               n_active, 0, grid, stream);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_closure_batch(int storage, const ClosureInst* insts, const int* bfirst, int n_active, int blocks,
                                int j, const ClosureNet* net, hipStream_t stream) {
  if (n_active < 1 || blocks < 1) return hipErrorInvalidValue;
  const int grid = std::min(blocks, 3 * device_cus());
  const ClosureGeo G{};
  const ClosureOdd odd{};
  switch (storage) {
    case STORE_FP64:
      return launch_infer_t<double, true, true>(nullptr, nullptr, nullptr, nullptr, G, net, odd, insts, bfirst,
                                                n_active, j, grid, stream);
    case STORE_FP32:
      return launch_infer_t<float, true, true>(nullptr, nullptr, nullptr, nullptr, G, net, odd, insts, bfirst,
                                               n_active, j, grid, stream);
    case STORE_BF16:
      return launch_infer_t<bf16, true, true>(nullptr, nullptr, nullptr, nullptr, G, net, odd, insts, bfirst,
                                              n_active, j, grid, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace starmap
