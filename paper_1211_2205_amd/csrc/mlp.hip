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
//   network : 128 -> 128 -> 128 -> 6, exact-erf GELU after the hidden layers;
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

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
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
template <typename T>
__global__ void __launch_bounds__(256) closure_samples_kernel(const T* __restrict__ U,
                                                              const typename ComputeOf<T>::type* __restrict__ decay,
                                                              const ClosureGeo G, const int* __restrict__ pts,
                                                              int count, float* __restrict__ feat,
                                                              float* __restrict__ targ) {
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
// Every workgroup holds the network in LDS and loops over blocks of 64
// evaluation points of the (nx + 1) x (ny + 1) index domain: gather and
// normalise the inputs, three MFMA layers (waves split the 128 hidden units;
// the last layer gives each wave 16 points), then nu * y / dx into the
// closure planes of the order-5 moments.
constexpr int CB = 64;               // evaluation points per block
constexpr int LDW = CLOSURE_IN + 8;  // LDS row of weights and activations (bf16)

template <typename T>
__global__ void __launch_bounds__(256) closure_infer_kernel(T* __restrict__ U,
                                                            const typename ComputeOf<T>::type* __restrict__ decay,
                                                            const ClosureGeo G, const ClosureNet* __restrict__ net) {
  using C = typename ComputeOf<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  uint16_t* W1 = reinterpret_cast<uint16_t*>(smem);  // [128][LDW]
  uint16_t* W2 = W1 + CLOSURE_HIDDEN * LDW;          // [128][LDW]
  uint16_t* W3 = W2 + CLOSURE_HIDDEN * LDW;          // [16][LDW], rows >= 6 zero
  uint16_t* Xa = W3 + 16 * LDW;                      // [64][LDW] inputs, then layer-2 activations
  uint16_t* Xb = Xa + CB * LDW;                      // [64][LDW] layer-1 activations
  C* nu_s = reinterpret_cast<C*>(Xb + CB * LDW);  // [64]
  C* part = nu_s + CB;                            // [4][64] partial sums of squares per wave
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  // weights: bf16 rows of 128, copied 16 bytes at a time
  for (int e = tid; e < (2 * CLOSURE_HIDDEN + 16) * (CLOSURE_IN / 8); e += 256) {
    const int row = e / (CLOSURE_IN / 8), c8 = (e % (CLOSURE_IN / 8)) * 8;
    const uint4 v = reinterpret_cast<const uint4*>(net->w)[e];
    *reinterpret_cast<uint4*>(&W1[row * LDW + c8]) = v;  // W1, W2, W3 rows are consecutive
  }
  float b1[2], b2[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    b1[j] = net->b1[32 * w + 16 * j + (lane & 15)];
    b2[j] = net->b2[32 * w + 16 * j + (lane & 15)];
  }
  const float b3 = net->b3[lane & 15];

  const int NXE = G.nx + 1, total = NXE * (G.ny + 1);
  const int nblk = (total + CB - 1) / CB;
  for (int blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    // 1. inputs: wave w gathers moments w, w + 4, w + 8 of point lane
    const int pt = blk * CB + lane;
    const bool live = pt < total;
    const int i = live ? pt % NXE : 0, j = live ? pt / NXE : 0;
    C v[3][9];
    C ss = C(0);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int p = w + 4 * t;
      if (p < CLOSURE_PLANES) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
          stencil_value(U, G, p, i, j, q % 3 - 1, q / 3 - 1, &v[t][q]);
          ss += v[t][q] * v[t][q];
        }
      }
    }
    __syncthreads();  // the previous block's reads of Xa, nu_s and part are done
    part[w * CB + lane] = ss;
    __syncthreads();
    const C nu = sqrt(((part[lane] + part[CB + lane]) + part[2 * CB + lane]) + part[3 * CB + lane]) + C(CLOSURE_EPS);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int p = w + 4 * t;
      if (p < CLOSURE_PLANES) {
#pragma unroll
        for (int q = 0; q < 9; ++q) Xa[lane * LDW + 9 * p + q] = uint16_t(bf16_bits(v[t][q] / nu));
      }
    }
    if (w == 3) {
      C fa, fs;
      sigma_inputs(decay, G, i, j, &fa, &fs);
      Xa[lane * LDW + 99] = uint16_t(bf16_bits(fa));
      Xa[lane * LDW + 100] = uint16_t(bf16_bits(fs));
      for (int q = 101; q < CLOSURE_IN; ++q) Xa[lane * LDW + q] = 0;
      nu_s[lane] = nu;
    }
    __syncthreads();

    // 2. hidden layers: wave w computes units [32 w, 32 w + 32) of all 64 points
    const int fk = 8 * (lane >> 4);
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
      const uint16_t* Xin = layer == 0 ? Xa : Xb;
      uint16_t* Xout = layer == 0 ? Xb : Xa;
      const uint16_t* Wl = layer == 0 ? W1 : W2;
      f32x4 acc[4][2];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < CLOSURE_IN; k0 += 32) {
        uint4 bfr[2];
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
          bfr[nj] = *reinterpret_cast<const uint4*>(&Wl[(32 * w + 16 * nj + (lane & 15)) * LDW + k0 + fk]);
#pragma unroll
        for (int mi = 0; mi < 4; ++mi) {
          const uint4 afr = *reinterpret_cast<const uint4*>(&Xin[(16 * mi + (lane & 15)) * LDW + k0 + fk]);
#pragma unroll
          for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = mfma16(afr, bfr[nj], acc[mi][nj]);
        }
      }
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = 16 * mi + 4 * (lane >> 4) + r;
            const int n = 32 * w + 16 * nj + (lane & 15);
            const float z = acc[mi][nj][r] + (layer == 0 ? b1[nj] : b2[nj]);
            Xout[m * LDW + n] = uint16_t(bf16_bits(gelu(z)));
          }
      __syncthreads();
    }

    // 3. output layer: wave w takes points [16 w, 16 w + 16), 16 outputs (6 used)
    f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < CLOSURE_IN; k0 += 32) {
      const uint4 afr = *reinterpret_cast<const uint4*>(&Xa[(16 * w + (lane & 15)) * LDW + k0 + fk]);
      const uint4 bfr = *reinterpret_cast<const uint4*>(&W3[(lane & 15) * LDW + k0 + fk]);
      y = mfma16(afr, bfr, y);
    }
    const int o = lane & 15;
    if (o < CLOSURE_OUT) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * w + 4 * (lane >> 4) + r;
        const int p2 = blk * CB + m;
        if (p2 >= total) continue;
        const int pi = p2 % NXE, pj = p2 / NXE;
        if (pi >= G.out_nx[o] || pj >= G.out_ny[o]) continue;
        const int X = internal_index(pi, G.out_nodex[o], G.px, G.nx);
        const int Y = internal_index(pj, G.out_nodey[o], G.py, G.ny);
        const C g = nu_s[m] * C(y[r] + b3) / C(G.dx);
        U[int64_t(G.q[o]) * G.plane_stride + int64_t(Y) * G.pitch + X] = from_c<T>(g);
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
                                  const int* pts, int count, float* feat, float* targ, hipStream_t stream) {
  const dim3 grid((count + 255) / 256);
  switch (storage) {
    case STORE_FP64:
      hipLaunchKernelGGL(closure_samples_kernel<double>, grid, dim3(256), 0, stream,
                         static_cast<const double*>(U), static_cast<const double*>(decay), G, pts, count, feat, targ);
      break;
    case STORE_FP32:
      hipLaunchKernelGGL(closure_samples_kernel<float>, grid, dim3(256), 0, stream,
                         static_cast<const float*>(U), static_cast<const float*>(decay), G, pts, count, feat, targ);
      break;
    case STORE_BF16:
      hipLaunchKernelGGL(closure_samples_kernel<bf16>, grid, dim3(256), 0, stream,
                         static_cast<const bf16*>(U), static_cast<const float*>(decay), G, pts, count, feat, targ);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t closure_infer_lds_bytes() {
  return size_t(2 * CLOSURE_HIDDEN + 16 + 2 * CB) * LDW * 2 + size_t(5 * CB) * 8;
}

namespace {
template <typename T>
hipError_t launch_infer_t(void* U, const void* decay, const ClosureGeo& G, const ClosureNet* net, int blocks,
                          hipStream_t stream) {
  using C = typename ComputeOf<T>::type;
  static bool attr = false;
  const size_t lds = closure_infer_lds_bytes();
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&closure_infer_kernel<T>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(closure_infer_kernel<T>, dim3(blocks), dim3(256), lds, stream, static_cast<T*>(U),
                     static_cast<const C*>(decay), G, net);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_closure_infer(int storage, void* U, const void* decay, const ClosureGeo& G, const ClosureNet* net,
                                hipStream_t stream) {
  // one workgroup per compute unit (the network fills most of its LDS), each
  // looping over blocks of points with the weights loaded once
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
  }
  const int total = (G.nx + 1) * (G.ny + 1);
  const int nblk = (total + CB - 1) / CB;
  const int blocks = std::min(nblk, cus);
  switch (storage) {
    case STORE_FP64: return launch_infer_t<double>(U, decay, G, net, blocks, stream);
    case STORE_FP32: return launch_infer_t<float>(U, decay, G, net, blocks, stream);
    case STORE_BF16: return launch_infer_t<bf16>(U, decay, G, net, blocks, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace starmap
