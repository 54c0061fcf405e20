// C ABI of the learned closure: loading a network into a P_5 solver, the
// closure kernel before every odd sweep, training samples from a high-order
// state, and the network trainer (forward, backward, Adam on the device).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/starmap.h"
#include "mlp.hpp"
#include "solver.hpp"

using namespace starmap;
using namespace starmap::detail;

namespace {

// (imag, l, m) of the closure's input moments (orders 4 and 5 of P_5, in
// moment order) and of its outputs (order 5).
struct Key {
  int imag, l, m;
};
const Key kInputs[CLOSURE_PLANES] = {{0, 4, 4}, {1, 4, 4}, {0, 4, 2}, {1, 4, 2}, {0, 4, 0}, {0, 5, 5},
                                     {1, 5, 5}, {0, 5, 3}, {1, 5, 3}, {0, 5, 1}, {1, 5, 1}};
const Key* const kOutputs = kInputs + 5;

int find_moment(const starmap_solver* s, const Key& key) {
  for (int k = 0; k < s->nmom; ++k)
    if (s->moms[k].imag == key.imag && s->moms[k].l == key.l && s->moms[k].m == key.m) return k;
  return -1;
}

uint16_t bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return uint16_t((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}

// offsets of the parameter blob
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + CLOSURE_HIDDEN * CLOSURE_IN;
constexpr int OFF_W2 = OFF_B1 + CLOSURE_HIDDEN;
constexpr int OFF_B2 = OFF_W2 + CLOSURE_HIDDEN * CLOSURE_HIDDEN;
constexpr int OFF_W3 = OFF_B2 + CLOSURE_HIDDEN;
constexpr int OFF_B3 = OFF_W3 + CLOSURE_OUT * CLOSURE_HIDDEN;
static_assert(OFF_B3 + CLOSURE_OUT == CLOSURE_PARAMS, "parameter blob layout");

}  // namespace

namespace starmap {
namespace detail {

int closure_geometry(const starmap_solver* s, ClosureGeo* g, bool with_terms) {
  std::memset(g, 0, sizeof(*g));
  if (s->N < 5) return fail(STARMAP_EINVAL, "the closure needs moments of orders 4 and 5");
  if (s->anisotropic) return fail(STARMAP_EINVAL, "the closure assumes isotropic scattering");
  for (int p = 0; p < CLOSURE_PLANES; ++p) {
    const int k = find_moment(s, kInputs[p]);
    if (k < 0) return fail(STARMAP_EINVAL, "closure input moment missing");
    g->k[p] = k;
    g->pnx[p] = points_x(s, s->moms[k].gx);
    g->pny[p] = points_y(s, s->moms[k].gy);
    g->nodex[p] = s->moms[k].gx == AXIS_NODE;
    g->nodey[p] = s->moms[k].gy == AXIS_NODE;
  }
  g->nx = s->nx;
  g->ny = s->ny;
  g->px = s->px;
  g->py = s->py;
  g->pitch = s->pitch;
  g->plane_stride = s->plane_stride;
  g->dx = s->dx;
  g->dy = s->dy;
  // sigma_a: the zeroth moment's decay plane; sigma_a + sigma_s: that of R_2^0 (G11)
  const int k20 = find_moment(s, {0, 2, 0});
  g->dk_a = s->dmap.dk[0];
  g->dk_t = s->dmap.dk[k20];
  if (s->dmap.plane_gx[g->dk_t] != AXIS_CELL || s->dmap.plane_gy[g->dk_t] != AXIS_CELL)
    return fail(STARMAP_EINVAL, "unexpected decay plane layout");
  for (int o = 0; o < CLOSURE_OUT; ++o) {
    const int k = find_moment(s, kOutputs[o]);
    g->q[o] = (s->qk.size() == size_t(s->nmom) && s->qk[k] >= 0) ? s->nmom + s->qk[k] : -1;
    g->out_nx[o] = points_x(s, s->moms[k].gx);
    g->out_ny[o] = points_y(s, s->moms[k].gy);
    g->out_nodex[o] = s->moms[k].gx == AXIS_NODE;
    g->out_nodey[o] = s->moms[k].gy == AXIS_NODE;
    if (!with_terms) continue;
    if (s->N < 6) return fail(STARMAP_EINVAL, "training targets need moments of order 6");
    const CouplingRow& r = s->rows[k];
    int n = 0;
    for (int t = 0; t < r.nx; ++t) {
      const int j = r.x[t].col;
      if (s->moms[j].l != 6) continue;
      if (n >= 4) return fail(STARMAP_EINVAL, "too many order-6 couplings");
      g->term[o][n++] = {j, 0, s->moms[j].gx == AXIS_CELL, 0, r.x[t].val};
    }
    for (int t = 0; t < r.ny; ++t) {
      const int j = r.y[t].col;
      if (s->moms[j].l != 6) continue;
      if (n >= 4) return fail(STARMAP_EINVAL, "too many order-6 couplings");
      g->term[o][n++] = {j, 1, s->moms[j].gy == AXIS_CELL, 0, r.y[t].val};
    }
    g->nterm[o] = n;
  }
  return STARMAP_OK;
}

int closure_plane_a(const starmap_solver* s) { return s->cgeo.k[5]; }
int closure_plane_b(const starmap_solver* s) { return s->nmom + s->qk[s->cgeo.k[5]]; }

int closure_odd_sweep(starmap_solver* s, double tau) {
  if (!s->closure_loaded) return fail(STARMAP_ESTATE, "learned closure: no network loaded (starmap_closure_load)");
  const size_t pb = s->plane_bytes_state();
  char* a = dptr(s, s->off_state + size_t(closure_plane_a(s)) * pb);
  char* b = dptr(s, s->off_state + size_t(closure_plane_b(s)) * pb);
  ClosureOdd odd = s->codd;
  odd.tau = tau;
  HIP_TRY(launch_closure_sweep(s->storage, dptr(s, s->off_state), s->c5_flip ? b : a, s->c5_flip ? a : b,
                               dptr(s, s->off_decay), s->cgeo, reinterpret_cast<const ClosureNet*>(dptr(s, s->off_net)),
                               odd, s->stream));
  s->c5_flip ^= 1;
  return STARMAP_OK;
}

int closure_settle(starmap_solver* s) {
  if (!s->c5_flip) return STARMAP_OK;
  const size_t pb = s->plane_bytes_state();
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_state + size_t(closure_plane_a(s)) * pb),
                         dptr(s, s->off_state + size_t(closure_plane_b(s)) * pb), CLOSURE_OUT * pb,
                         hipMemcpyDeviceToDevice, s->stream));
  s->c5_flip = 0;
  return STARMAP_OK;
}

int closure_before_odd(starmap_solver* s) {
  if (!s->closure_loaded) return fail(STARMAP_ESTATE, "learned closure: no network loaded (starmap_closure_load)");
  HIP_TRY(launch_closure_infer(s->storage, dptr(s, s->off_state), dptr(s, s->off_decay), s->cgeo,
                               reinterpret_cast<const ClosureNet*>(dptr(s, s->off_net)), s->stream));
  return STARMAP_OK;
}

}  // namespace detail
}  // namespace starmap

// ------------------------------------------------------------ trainer object
struct starmap_mlp {
  hipStream_t stream = nullptr;
  int max_batch = 0;
  void* mem = nullptr;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  float *Z1 = nullptr, *A1 = nullptr, *Z2 = nullptr, *A2 = nullptr, *Y = nullptr, *dY = nullptr;
  float *dZ1 = nullptr, *dZ2 = nullptr, *gpart = nullptr, *cpart = nullptr;
  double *lpart = nullptr, *loss = nullptr;
  int splits = 1;
  int64_t t = 0;  // Adam steps taken
};

namespace {

constexpr int kMaxSplits = 64;
constexpr int kLossBlocks = 256;

int mlp_forward(starmap_mlp* n, const float* X, int B) {
  const float* P = n->params;
  auto layer = [&](const float* A, const float* W, int N, const float* bias, int mode, float* out, float* out2,
                   int ldo) -> int {
    GemmArgs g{A, CLOSURE_IN, 1, W, 1, CLOSURE_IN, n->gpart, B, N, CLOSURE_IN, 1 << 30};
    EpiArgs e{n->gpart, 1, B, N, bias, mode, nullptr, 0, out, ldo, out2};
    HIP_TRY(launch_gemm(g, 1, e, n->stream));
    return STARMAP_OK;
  };
  int rc = layer(X, P + OFF_W1, CLOSURE_HIDDEN, P + OFF_B1, EPI_GELU, n->Z1, n->A1, CLOSURE_HIDDEN);
  if (!rc) rc = layer(n->A1, P + OFF_W2, CLOSURE_HIDDEN, P + OFF_B2, EPI_GELU, n->Z2, n->A2, CLOSURE_HIDDEN);
  if (!rc) rc = layer(n->A2, P + OFF_W3, CLOSURE_OUT, P + OFF_B3, EPI_STORE, n->Y, nullptr, CLOSURE_OUT);
  return rc;
}

// weight gradient G (M x 128) = D^T A over the batch: D (B x M), A (B x 128)
int mlp_weight_grad(starmap_mlp* n, const float* D, int M, const float* A, int B, float* G) {
  int splits = std::min(kMaxSplits, std::max(1, B / 256));
  int kchunk = ((B + splits - 1) / splits + 31) / 32 * 32;
  splits = (B + kchunk - 1) / kchunk;
  GemmArgs g{D, 1, M, A, CLOSURE_HIDDEN, 1, n->gpart, M, CLOSURE_HIDDEN, B, kchunk};
  EpiArgs e{n->gpart, splits, M, CLOSURE_HIDDEN, nullptr, EPI_STORE, nullptr, 0, G, CLOSURE_HIDDEN, nullptr};
  HIP_TRY(launch_gemm(g, splits, e, n->stream));
  return STARMAP_OK;
}

int mlp_backward(starmap_mlp* n, const float* X, const float* T, int B) {
  const float* P = n->params;
  float* G = n->grads;
  HIP_TRY(launch_mse(n->Y, T, int64_t(B) * CLOSURE_OUT, n->dY, n->lpart, kLossBlocks, n->loss, n->stream));
  int rc = mlp_weight_grad(n, n->dY, CLOSURE_OUT, n->A2, B, G + OFF_W3);
  if (rc) return rc;
  HIP_TRY(launch_colsum(n->dY, B, CLOSURE_OUT, CLOSURE_OUT, n->cpart, G + OFF_B3, n->stream));
  {  // dZ2 = (dY W3) * gelu'(Z2)
    GemmArgs g{n->dY, CLOSURE_OUT, 1, P + OFF_W3, CLOSURE_HIDDEN, 1, n->gpart, B, CLOSURE_HIDDEN, CLOSURE_OUT, 1 << 30};
    EpiArgs e{n->gpart, 1, B, CLOSURE_HIDDEN, nullptr, EPI_GELU_GRAD, n->Z2, CLOSURE_HIDDEN, n->dZ2, CLOSURE_HIDDEN,
              nullptr};
    HIP_TRY(launch_gemm(g, 1, e, n->stream));
  }
  rc = mlp_weight_grad(n, n->dZ2, CLOSURE_HIDDEN, n->A1, B, G + OFF_W2);
  if (rc) return rc;
  HIP_TRY(launch_colsum(n->dZ2, B, CLOSURE_HIDDEN, CLOSURE_HIDDEN, n->cpart, G + OFF_B2, n->stream));
  {  // dZ1 = (dZ2 W2) * gelu'(Z1)
    GemmArgs g{n->dZ2, CLOSURE_HIDDEN, 1, P + OFF_W2, CLOSURE_HIDDEN, 1, n->gpart, B, CLOSURE_HIDDEN,
               CLOSURE_HIDDEN, 1 << 30};
    EpiArgs e{n->gpart, 1, B, CLOSURE_HIDDEN, nullptr, EPI_GELU_GRAD, n->Z1, CLOSURE_HIDDEN, n->dZ1, CLOSURE_HIDDEN,
              nullptr};
    HIP_TRY(launch_gemm(g, 1, e, n->stream));
  }
  rc = mlp_weight_grad(n, n->dZ1, CLOSURE_HIDDEN, X, B, G + OFF_W1);
  if (rc) return rc;
  HIP_TRY(launch_colsum(n->dZ1, B, CLOSURE_HIDDEN, CLOSURE_HIDDEN, n->cpart, G + OFF_B1, n->stream));
  return STARMAP_OK;
}

int check_batch(const starmap_mlp* n, int B) {
  if (!n) return fail(STARMAP_EINVAL, "trainer is NULL");
  if (B < 1 || B > n->max_batch) return fail(STARMAP_EINVAL, "batch size out of range");
  return STARMAP_OK;
}

}  // namespace

extern "C" {

int starmap_closure_load(starmap_solver* s, const float* w, size_t count) {
  if (!s || !w) return fail(STARMAP_EINVAL, "bad arguments");
  if (!s->closure) return fail(STARMAP_ESTATE, "the solver was not created with STARMAP_CLOSURE_LEARNED");
  if (count != size_t(CLOSURE_PARAMS)) return fail(STARMAP_EINVAL, "closure weights: wrong parameter count");
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(w[i])) return fail(STARMAP_EINVAL, "closure weights: non-finite value");
  int rc = ensure_device(s);
  if (rc) return rc;
  rc = closure_geometry(s, &s->cgeo, false);
  if (rc) return rc;
  auto net = std::make_unique<ClosureNet>();
  std::memset(net.get(), 0, sizeof(ClosureNet));
  for (int r = 0; r < CLOSURE_HIDDEN; ++r)
    for (int c = 0; c < CLOSURE_IN; ++c) {
      net->w[r * CLOSURE_IN + c] = bf16_rne(w[OFF_W1 + r * CLOSURE_IN + c]);
      net->w[(CLOSURE_HIDDEN + r) * CLOSURE_IN + c] = bf16_rne(w[OFF_W2 + r * CLOSURE_HIDDEN + c]);
    }
  for (int r = 0; r < CLOSURE_OUT; ++r)
    for (int c = 0; c < CLOSURE_HIDDEN; ++c)
      net->w[(2 * CLOSURE_HIDDEN + r) * CLOSURE_IN + c] = bf16_rne(w[OFF_W3 + r * CLOSURE_HIDDEN + c]);
  std::memcpy(net->b1, w + OFF_B1, sizeof(net->b1));
  std::memcpy(net->b2, w + OFF_B2, sizeof(net->b2));
  std::memcpy(net->b3, w + OFF_B3, CLOSURE_OUT * sizeof(float));
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_net), net.get(), sizeof(ClosureNet), hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  // the odd rows of the fused closure sweep
  for (int o = 0; o < CLOSURE_OUT; ++o)
    if (s->cgeo.k[5 + o] != s->cgeo.k[5] + o || s->qk[s->cgeo.k[5 + o]] != s->qk[s->cgeo.k[5]] + o)
      return fail(STARMAP_EINVAL, "closure: order-5 planes are not consecutive");
  std::memset(&s->codd, 0, sizeof(s->codd));
  int q = 0;
  for (int k = 0; k < s->nmom; ++k) {
    const MomentInfo& mk = s->moms[k];
    if (mk.l % 2 == 0) continue;
    if (q >= CLOSURE_ODD_ROWS) return fail(STARMAP_EINVAL, "closure: too many odd moments");
    ClosureOddRow& r = s->codd.r[q++];
    r.k = k;
    r.node_x = mk.gx == AXIS_NODE;
    r.dk = s->dmap.dk[k];
    r.o = mk.l == 5 ? k - s->cgeo.k[5] : -1;
    r.src = (r.o < 0 && s->qk[k] >= 0) ? s->nmom + s->qk[k] : -1;
    const CouplingRow& cr = s->rows[k];
    r.nx = cr.nx;
    r.ny = cr.ny;
    for (int t = 0; t < cr.nx; ++t) {
      r.xk[t] = cr.x[t].col;
      r.xcell[t] = s->moms[cr.x[t].col].gx == AXIS_CELL;
      r.xc[t] = -cr.x[t].val / s->dx;
    }
    for (int t = 0; t < cr.ny; ++t) {
      r.yk[t] = cr.y[t].col;
      r.ycell[t] = s->moms[cr.y[t].col].gy == AXIS_CELL;
      r.yc[t] = -cr.y[t].val / s->dy;
    }
  }
  if (q != CLOSURE_ODD_ROWS) return fail(STARMAP_EINVAL, "closure: unexpected number of odd moments");
  s->closure_w.assign(w, w + count);
  s->closure_loaded = true;
  return STARMAP_OK;
}

int starmap_closure_set_fused(starmap_solver* s, int32_t enable) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (!s->closure) return fail(STARMAP_ESTATE, "the solver was not created with STARMAP_CLOSURE_LEARNED");
  int rc = closure_settle(s);
  if (rc) return rc;
  s->closure_fused = enable != 0;
  ++s->graph_version;  // the launch sequence changes
  return STARMAP_OK;
}

namespace {
// Closure inputs (and, with targets, the order-6 flux) at cells of a solver's
// current state; nu_out and targets may be null.
int closure_points(starmap_solver* s, const int32_t* points, int32_t count, float* features, float* targets,
                   float* nu_out) {
  if (count == 0) return STARMAP_OK;
  for (int32_t i = 0; i < count; ++i)
    if (points[2 * i] < 0 || points[2 * i] >= s->nx || points[2 * i + 1] < 0 || points[2 * i + 1] >= s->ny)
      return fail(STARMAP_EINVAL, "sample point outside the cells");
  ClosureGeo g;
  int rc = closure_geometry(s, &g, targets != nullptr);
  if (rc) return rc;
  rc = ensure_device(s);
  if (rc) return rc;
  if (!s->materials_ready) {
    rc = ensure_materials(s, s->t + 0.5 * s->dt);
    if (rc) return rc;
  }
  const size_t bytes = size_t(count) * 2 * sizeof(int32_t);
  if (bytes > s->sample_cap) {
    if (s->sample_buf) HIP_TRY(hipFree(s->sample_buf));
    s->sample_buf = nullptr;
    s->sample_cap = 0;
    HIP_TRY(hipMalloc(&s->sample_buf, bytes));
    s->sample_cap = bytes;
  }
  HIP_TRY(hipMemcpyAsync(s->sample_buf, points, bytes, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(launch_closure_samples(s->storage, dptr(s, s->off_state), dptr(s, s->off_decay), g,
                                 static_cast<const int*>(s->sample_buf), count, features, targets, nu_out,
                                 s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return STARMAP_OK;
}
}  // namespace

int starmap_closure_samples(starmap_solver* s, const int32_t* points, int32_t count, float* features,
                            float* targets) {
  if (!s || !points || !features || !targets || count < 0) return fail(STARMAP_EINVAL, "bad arguments");
  return closure_points(s, points, count, features, targets, nullptr);
}

int starmap_closure_features(starmap_solver* s, const int32_t* points, int32_t count, float* features,
                             float* nu) {
  if (!s || !points || !features || count < 0) return fail(STARMAP_EINVAL, "bad arguments");
  return closure_points(s, points, count, features, nullptr, nu);
}

int starmap_mlp_create(int32_t max_batch, void* hip_stream, starmap_mlp** out) {
  if (!out) return fail(STARMAP_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 24)) return fail(STARMAP_EINVAL, "max_batch out of range");
  auto n = std::make_unique<starmap_mlp>();
  n->stream = static_cast<hipStream_t>(hip_stream);
  n->max_batch = max_batch;
  const size_t P = align256(size_t(CLOSURE_PARAMS) * 4);
  const size_t act = align256(size_t(max_batch) * CLOSURE_HIDDEN * 4);
  const size_t out6 = align256(size_t(max_batch) * CLOSURE_OUT * 4);
  const size_t gp = align256(std::max(size_t(kMaxSplits) * CLOSURE_HIDDEN * CLOSURE_HIDDEN,
                                      size_t(max_batch) * CLOSURE_HIDDEN) * 4);
  const size_t cp = align256(size_t(colsum_part_floats(max_batch, CLOSURE_HIDDEN)) * 4);
  const size_t lp = align256(size_t(kLossBlocks + 1) * 8);
  const size_t total = 4 * P + 6 * act + 2 * out6 + gp + cp + lp;
  HIP_TRY(hipMalloc(&n->mem, total));
  HIP_TRY(hipMemsetAsync(n->mem, 0, total, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  char* p = static_cast<char*>(n->mem);
  auto take = [&](size_t b) { char* r = p; p += b; return r; };
  n->params = reinterpret_cast<float*>(take(P));
  n->grads = reinterpret_cast<float*>(take(P));
  n->m = reinterpret_cast<float*>(take(P));
  n->v = reinterpret_cast<float*>(take(P));
  n->Z1 = reinterpret_cast<float*>(take(act));
  n->A1 = reinterpret_cast<float*>(take(act));
  n->Z2 = reinterpret_cast<float*>(take(act));
  n->A2 = reinterpret_cast<float*>(take(act));
  n->dZ1 = reinterpret_cast<float*>(take(act));
  n->dZ2 = reinterpret_cast<float*>(take(act));
  n->Y = reinterpret_cast<float*>(take(out6));
  n->dY = reinterpret_cast<float*>(take(out6));
  n->gpart = reinterpret_cast<float*>(take(gp));
  n->cpart = reinterpret_cast<float*>(take(cp));
  n->lpart = reinterpret_cast<double*>(take(lp));
  n->loss = n->lpart + kLossBlocks;
  *out = n.release();
  return STARMAP_OK;
}

void starmap_mlp_destroy(starmap_mlp* n) {
  if (!n) return;
  if (n->mem) {
    (void)hipStreamSynchronize(n->stream);
    (void)hipFree(n->mem);
  }
  delete n;
}

int starmap_mlp_set_params(starmap_mlp* n, const float* w, size_t count) {
  if (!n || !w) return fail(STARMAP_EINVAL, "bad arguments");
  if (count != size_t(CLOSURE_PARAMS)) return fail(STARMAP_EINVAL, "wrong parameter count");
  HIP_TRY(hipMemcpyAsync(n->params, w, count * 4, hipMemcpyHostToDevice, n->stream));
  HIP_TRY(hipMemsetAsync(n->m, 0, count * 4, n->stream));
  HIP_TRY(hipMemsetAsync(n->v, 0, count * 4, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  n->t = 0;
  return STARMAP_OK;
}

int starmap_mlp_get_params(const starmap_mlp* n, float* w, size_t count) {
  if (!n || !w) return fail(STARMAP_EINVAL, "bad arguments");
  if (count != size_t(CLOSURE_PARAMS)) return fail(STARMAP_EINVAL, "wrong parameter count");
  HIP_TRY(hipMemcpyAsync(w, n->params, count * 4, hipMemcpyDeviceToHost, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  return STARMAP_OK;
}

int starmap_mlp_forward(starmap_mlp* n, const float* x, int32_t batch, float* y) {
  int rc = check_batch(n, batch);
  if (rc) return rc;
  if (!x || !y) return fail(STARMAP_EINVAL, "bad arguments");
  rc = mlp_forward(n, x, batch);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(y, n->Y, size_t(batch) * CLOSURE_OUT * 4, hipMemcpyDeviceToDevice, n->stream));
  return STARMAP_OK;
}

int starmap_mlp_gradients(starmap_mlp* n, const float* x, const float* t, int32_t batch, float* grad_host,
                          double* loss) {
  int rc = check_batch(n, batch);
  if (rc) return rc;
  if (!x || !t) return fail(STARMAP_EINVAL, "bad arguments");
  rc = mlp_forward(n, x, batch);
  if (!rc) rc = mlp_backward(n, x, t, batch);
  if (rc) return rc;
  if (grad_host)
    HIP_TRY(hipMemcpyAsync(grad_host, n->grads, size_t(CLOSURE_PARAMS) * 4, hipMemcpyDeviceToHost, n->stream));
  if (loss) HIP_TRY(hipMemcpyAsync(loss, n->loss, 8, hipMemcpyDeviceToHost, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  return STARMAP_OK;
}

int starmap_mlp_train_step(starmap_mlp* n, const float* x, const float* t, int32_t batch, double lr, double* loss) {
  int rc = check_batch(n, batch);
  if (rc) return rc;
  if (!x || !t || !(lr > 0.0)) return fail(STARMAP_EINVAL, "bad arguments");
  rc = mlp_forward(n, x, batch);
  if (!rc) rc = mlp_backward(n, x, t, batch);
  if (rc) return rc;
  n->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, double(n->t)), c2 = 1.0 - std::pow(b2, double(n->t));
  HIP_TRY(launch_adam(n->params, n->grads, n->m, n->v, CLOSURE_PARAMS, float(lr), float(b1), float(b2), 1e-8f,
                      float(c1), float(c2), n->stream));
  if (loss) {
    HIP_TRY(hipMemcpyAsync(loss, n->loss, 8, hipMemcpyDeviceToHost, n->stream));
    HIP_TRY(hipStreamSynchronize(n->stream));
  }
  return STARMAP_OK;
}

int starmap_mlp_adam_step(starmap_mlp* n, const float* grad_host, double lr) {
  if (!n || !grad_host || !(lr > 0.0)) return fail(STARMAP_EINVAL, "bad arguments");
  HIP_TRY(hipMemcpyAsync(n->grads, grad_host, size_t(CLOSURE_PARAMS) * 4, hipMemcpyHostToDevice, n->stream));
  n->t += 1;
  const double b1 = 0.9, b2 = 0.999;
  const double c1 = 1.0 - std::pow(b1, double(n->t)), c2 = 1.0 - std::pow(b2, double(n->t));
  HIP_TRY(launch_adam(n->params, n->grads, n->m, n->v, CLOSURE_PARAMS, float(lr), float(b1), float(b2), 1e-8f,
                      float(c1), float(c2), n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  return STARMAP_OK;
}

}  // extern "C"
