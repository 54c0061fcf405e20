// C ABI of the staggered-grid P_N solver: problem setup, host sampling of the
// fields, device workspace, time stepping, checkpoints and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/starmap.h"
#include "kernels.hpp"
#include "plan.hpp"
#include "solver.hpp"

using namespace starmap;

namespace starmap {
namespace detail {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

}  // namespace detail
}  // namespace starmap

using namespace starmap::detail;

namespace starmap {
namespace detail {

int points_x(const starmap_solver* s, int gx) { return gx == AXIS_CELL ? s->nx : s->nx + 1 - s->px; }
int points_y(const starmap_solver* s, int gy) { return gy == AXIS_CELL ? s->ny : s->ny + 1 - s->py; }

// Internal storage index of public index a along an axis: nodes of a periodic
// axis are stored modulo n (node n, the last public node, lands on index 0).
int internal_x(const starmap_solver* s, int gx, int a) {
  return (gx == AXIS_NODE && s->px) ? (a + 1) % s->nx : a;
}
int internal_y(const starmap_solver* s, int gy, int b) {
  return (gy == AXIS_NODE && s->py) ? (b + 1) % s->ny : b;
}

void grid_coords(const starmap_solver* s, int gx, int gy, std::vector<double>& X, std::vector<double>& Y) {
  const int nxk = points_x(s, gx), nyk = points_y(s, gy);
  X.resize(size_t(nxk) * nyk);
  Y.resize(size_t(nxk) * nyk);
  for (int b = 0; b < nyk; ++b) {
    const double y = gy == AXIS_CELL ? s->prob.ax[2] + (b + 0.5) * s->dy : s->prob.ax[2] + (b + s->py) * s->dy;
    for (int a = 0; a < nxk; ++a) {
      const double x = gx == AXIS_CELL ? s->prob.ax[0] + (a + 0.5) * s->dx : s->prob.ax[0] + (a + s->px) * s->dx;
      X[size_t(b) * nxk + a] = x;
      Y[size_t(b) * nxk + a] = y;
    }
  }
}

// Sample a field on grid (gx, gy) at time t (public layout); zero if unset.
int sample(const starmap_solver* s, const FieldSource& f, int gx, int gy, double t, std::vector<double>& out) {
  const int g = grid_id(gx, gy);
  const size_t n = size_t(points_x(s, gx)) * points_y(s, gy);
  if (f.has_array[g]) {
    out = f.arrays[g];
    return STARMAP_OK;
  }
  out.assign(n, 0.0);
  if (!f.fn && f.terms.empty()) return STARMAP_OK;
  std::vector<double> X, Y;
  grid_coords(s, gx, gy, X, Y);
  if (!f.terms.empty()) {  // sum a_i(t) g_i(x, y)
    std::vector<double> g(n);
    for (const FieldTerm& term : f.terms) {
      if (term.space(term.space_ctx, 0.0, int64_t(n), X.data(), Y.data(), g.data()) != 0)
        return fail(STARMAP_EINVAL, "field callback reported an error");
      const double a = term.time(term.time_ctx, t);
      for (size_t i = 0; i < n; ++i) out[i] += a * g[i];
    }
    return STARMAP_OK;
  }
  if (f.fn(f.ctx, t, int64_t(n), X.data(), Y.data(), out.data()) != 0)
    return fail(STARMAP_EINVAL, "field callback reported an error");
  return STARMAP_OK;
}

// The spatial part g of one term of a separable field on grid (gx, gy), or
// (term = -1) the whole time-independent field.
int sample_basis(const starmap_solver* s, const FieldSource& f, int term, int gx, int gy, std::vector<double>& out) {
  if (term < 0) return sample(s, f, gx, gy, 0.0, out);
  const size_t n = size_t(points_x(s, gx)) * points_y(s, gy);
  out.assign(n, 0.0);
  std::vector<double> X, Y;
  grid_coords(s, gx, gy, X, Y);
  const FieldTerm& t = f.terms[size_t(term)];
  if (t.space(t.space_ctx, 0.0, int64_t(n), X.data(), Y.data(), out.data()) != 0)
    return fail(STARMAP_EINVAL, "field callback reported an error");
  return STARMAP_OK;
}

template <typename T>
void to_type(double v, T* out) { *out = T(v); }
void to_type(double v, uint16_t* out) {
  float f = float(v);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) { *out = uint16_t((u >> 16) | 0x40u); return; }
  u += 0x7FFFu + ((u >> 16) & 1u);
  *out = uint16_t(u >> 16);
}
double from_type(double v) { return v; }
double from_type(float v) { return v; }
double from_type(uint16_t v) {
  uint32_t u = uint32_t(v) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Scatter a public-layout plane into a padded internal plane of type T.
template <typename T>
void scatter_plane(const starmap_solver* s, int gx, int gy, const double* vals, std::vector<T>& buf) {
  buf.assign(size_t(s->plane_stride), T(0));
  const int nxk = points_x(s, gx), nyk = points_y(s, gy);
  for (int b = 0; b < nyk; ++b) {
    const int Yi = internal_y(s, gy, b);
    for (int a = 0; a < nxk; ++a) {
      const int Xi = internal_x(s, gx, a);
      to_type(vals[size_t(b) * nxk + a], &buf[size_t(Yi) * s->pitch + Xi]);
    }
  }
}

template <typename T>
void gather_plane(const starmap_solver* s, int gx, int gy, const T* buf, double* out) {
  const int nxk = points_x(s, gx), nyk = points_y(s, gy);
  for (int b = 0; b < nyk; ++b) {
    const int Yi = internal_y(s, gy, b);
    for (int a = 0; a < nxk; ++a) {
      out[size_t(b) * nxk + a] = from_type(buf[size_t(Yi) * s->pitch + internal_x(s, gx, a)]);
    }
  }
}

int upload_plane(starmap_solver* s, void* dst, int gx, int gy, const double* vals, bool compute_type) {
  const int kind = compute_type ? (s->storage == STORE_FP64 ? 0 : 1) : s->storage;
  if (kind == STORE_FP64) {
    std::vector<double> buf;
    scatter_plane(s, gx, gy, vals, buf);
    HIP_TRY(hipMemcpyAsync(dst, buf.data(), buf.size() * 8, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else if (kind == STORE_FP32) {
    std::vector<float> buf;
    scatter_plane(s, gx, gy, vals, buf);
    HIP_TRY(hipMemcpyAsync(dst, buf.data(), buf.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else {
    std::vector<uint16_t> buf;
    scatter_plane(s, gx, gy, vals, buf);
    HIP_TRY(hipMemcpyAsync(dst, buf.data(), buf.size() * 2, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return STARMAP_OK;
}

char* dptr(const starmap_solver* s, size_t off) { return static_cast<char*>(s->dev) + off; }

// m-range widths the autotuner tries (the compiled tiles stage up to ten
// planes per order in registers, enough for ranges of up to eight indices)
constexpr int kDefaultChunkWidth = 8;
constexpr int kChunkWidths[] = {4, 6, 8};

size_t program_bytes(const SweepProgram& pr, size_t csize) {
  return align256(pr.chunks.size() * 16) + align256(pr.orders.size() * 16) + align256(pr.loads.size() * 16) +
         align256(pr.rows.size() * 64) + align256(pr.coefs.size() * csize);
}

// Time-separable fields: every decay plane, then every physical source plane,
// as a signed sum of basis planes (one per (field, term, grid); a
// time-independent field is one basis plane with factor 1).
// Filter damping of the decay plane of order l (l = -1: the zeroth moment).
double order_damping(const starmap_solver* s, int l) {
  if (s->damping.empty()) return 0.0;
  return s->damping[size_t(l < 0 ? 0 : l)];
}

void plan_separable(starmap_solver* s) {
  s->basis.clear();
  s->time_terms.clear();
  s->comb_tab.clear();
  s->basis_ready = false;
  s->static_done = false;
  auto has_terms = [](const FieldSource& f) { return !f.terms.empty(); };
  bool any = has_terms(s->absorption) || has_terms(s->scattering);
  for (auto& kv : s->scattering_order) any = any || has_terms(kv.second);
  for (auto& kv : s->source) any = any || has_terms(kv.second);
  s->separable = any;
  s->nbasis = 0;
  if (!any) return;
  std::map<std::pair<const FieldSource*, int>, int> tidx;
  std::map<std::tuple<const FieldSource*, int, int>, int> bidx;
  std::vector<int32_t> first(1, 0), entries;
  bool dynamic = false;
  auto add = [&](const FieldSource& f, int sign, int gx, int gy) {
    if (!f.set()) return;
    const int nt = int(f.terms.size());
    for (int t = (nt ? 0 : -1); t < (nt ? nt : 0); ++t) {
      auto key = std::make_tuple(&f, t, grid_id(gx, gy));
      auto it = bidx.find(key);
      if (it == bidx.end()) {
        it = bidx.emplace(key, int(s->basis.size())).first;
        s->basis.push_back({&f, t, gx, gy});
      }
      int ti = -1;
      if (t >= 0) {
        auto jt = tidx.find({&f, t});
        if (jt == tidx.end()) {
          jt = tidx.emplace(std::make_pair(&f, t), int(s->time_terms.size())).first;
          s->time_terms.push_back(f.terms[size_t(t)]);
        }
        ti = jt->second;
        dynamic = true;
      }
      entries.insert(entries.end(), {it->second, ti, sign});
    }
  };
  std::vector<int32_t> lists[4];
  s->comb_cst.clear();
  auto close_output = [&](int dst, int which, double cst) {
    const int o = int(first.size()) - 1;
    first.push_back(int32_t(entries.size() / 3));
    s->comb_cst.push_back(cst);
    lists[which].insert(lists[which].end(), {o, dst});
    if (dynamic) lists[which + 1].insert(lists[which + 1].end(), {o, dst});
    dynamic = false;
  };
  // decay: sigma_a (zeroth order), sigma_a + sigma_s0 - sigma_sl (order l >= 1)
  for (int p = 0; p < s->dmap.nplanes; ++p) {
    const int gx = s->dmap.plane_gx[p], gy = s->dmap.plane_gy[p], l = s->dmap.plane_l[p];
    add(s->absorption, 1, gx, gy);
    if (l >= 1) {
      add(s->scattering, 1, gx, gy);
      auto it = s->scattering_order.find(l);
      if (s->anisotropic && it != s->scattering_order.end()) add(it->second, -1, gx, gy);
    }
    close_output(p, 0, order_damping(s, l));
  }
  for (auto& kv : s->source) {
    const int k = kv.first;
    if (s->qk[k] < 0) continue;
    add(kv.second, 1, s->moms[k].gx, s->moms[k].gy);
    close_output(s->qk[k], 2, 0.0);
  }
  s->nbasis = int(s->basis.size());
  auto& tab = s->comb_tab;
  s->tab_first = 0;
  tab.insert(tab.end(), first.begin(), first.end());
  s->tab_entries = int(tab.size());
  tab.insert(tab.end(), entries.begin(), entries.end());
  for (int w = 0; w < 4; ++w) {
    s->tab_list[w] = int(tab.size());
    s->nlist[w] = int(lists[w].size() / 2);
    tab.insert(tab.end(), lists[w].begin(), lists[w].end());
  }
}

// Table of the parity-fused pass, one 16-int record per moment in processing
// order (the moments with odd parity, then those with even parity):
// {gx, gy, decay plane, source plane}, {k, reload, k P, 0}, four x and four y
// couplings as LDS offsets j P - o and j P - o R (P, R: the pass's staged
// plane and row; o = 1 when moment j is cell centred along the axis).  reload = 1 when the decay plane differs from the one the previous
// moment of the same parity and x grid class used.  Coupling lists are padded
// to four entries with coefficient 0 on a column of the other parity.  Eight
// coefficients per record, the separate sweeps' own (-M(k, j) / dx and
// -M(k, j) / dy in the rows' order).
void plan_fused(starmap_solver* s) {
  std::vector<int32_t> odd, even;
  for (int k = 0; k < s->nmom; ++k) (s->moms[k].gx == s->moms[k].gy ? even : odd).push_back(k);
  std::vector<int32_t> order = odd;
  order.insert(order.end(), even.begin(), even.end());
  s->ftab.assign(size_t(s->nmom) * 16, 0);
  s->fcoef.assign(size_t(s->nmom) * 8, 0.0);
  int last_dk[2][2] = {{-1, -1}, {-1, -1}};  // [parity][x grid class]
  for (int q = 0; q < s->nmom; ++q) {
    const int k = order[q];
    const auto& mk = s->moms[k];
    const int parity = mk.gx == mk.gy ? 1 : 0;
    int32_t* t = &s->ftab[size_t(q) * 16];
    double* cf = &s->fcoef[size_t(q) * 8];
    const CouplingRow& r = s->rows[k];
    t[0] = mk.gx;
    t[1] = mk.gy;
    t[2] = s->dmap.dk[k];
    t[3] = s->qk[k];
    t[4] = k;
    t[6] = k * kFusedPlane;
    int& last = last_dk[parity][mk.gx == 1 ? 1 : 0];
    t[5] = t[2] != last ? 1 : 0;
    last = t[2];
    const std::vector<int32_t>& others = parity ? odd : even;
    const int other = others.empty() ? k : others[0];  // P_0 has no couplings
    for (int i = 0; i < 4; ++i) {
      const int jx = i < r.nx ? r.x[i].col : (r.nx ? r.x[0].col : other);
      const int jy = i < r.ny ? r.y[i].col : (r.ny ? r.y[0].col : other);
      t[8 + i] = jx * kFusedPlane - (s->moms[jx].gx == 1 ? 1 : 0);
      t[12 + i] = jy * kFusedPlane - (s->moms[jy].gy == 1 ? kFusedRow : 0);
      cf[i] = i < r.nx ? -r.x[i].val / s->dx : 0.0;
      cf[4 + i] = i < r.ny ? -r.y[i].val / s->dy : 0.0;
    }
  }
  for (int d = 0; d < s->dmap.nplanes; ++d) s->ftab.insert(s->ftab.end(), {s->dmap.plane_gx[d], s->dmap.plane_gy[d], 0, 0});
  s->fnodd = int(odd.size());
  s->fused_ready = false;
}

int upload_fused(starmap_solver* s) {
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_ftab), s->ftab.data(), s->ftab.size() * 4, hipMemcpyHostToDevice,
                         s->stream));
  if (s->csize == 8) {
    HIP_TRY(hipMemcpyAsync(dptr(s, s->off_ftab + align256(s->ftab.size() * 4)), s->fcoef.data(),
                           s->fcoef.size() * 8, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  } else {
    std::vector<float> cf(s->fcoef.begin(), s->fcoef.end());
    HIP_TRY(hipMemcpyAsync(dptr(s, s->off_ftab + align256(s->ftab.size() * 4)), cf.data(), cf.size() * 4,
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  s->fused_ready = true;
  return STARMAP_OK;
}

// One parity-fused pass: S^o_tau_odd then S^e_tau_even, state read from the
// buffer at off_in and written to the one at off_out.
int fused_pass(starmap_solver* s, size_t off_in, size_t off_out, double tau_odd, double tau_even) {
  if (!s->fused_ready) {
    int rc = upload_fused(s);
    if (rc) return rc;
  }
  FusedArgs f;
  f.uin = dptr(s, off_in);
  f.uout = dptr(s, off_out);
  f.src = dptr(s, s->off_src);
  f.decay = dptr(s, s->off_decay);
  f.tab = reinterpret_cast<const int*>(dptr(s, s->off_ftab));
  f.coef = dptr(s, s->off_ftab + align256(s->ftab.size() * 4));
  f.ps = uint32_t(s->plane_stride);
  f.pitch = s->pitch;
  f.nx = s->nx;
  f.ny = s->ny;
  f.px = s->px;
  f.py = s->py;
  f.ntx = (s->nx + 1 + kFusedTX - 1) / kFusedTX;
  f.nty = (s->ny + 1 + kFusedTY - 1) / kFusedTY;
  f.nmom = s->nmom;
  f.nodd = s->fnodd;
  f.nd = s->dmap.nplanes;
  f.tau_odd = tau_odd;
  f.tau_even = tau_even;
  HIP_TRY(launch_fused(s->storage, f, s->stream));
  return STARMAP_OK;
}

void layout(starmap_solver* s) {
  // decay planes and source planes
  s->dmap = decay_map(s->N, s->anisotropic);
  s->qk.assign(s->nmom, -1);
  s->nsrc = 0;
  for (auto& kv : s->source)
    if (kv.second.set()) s->qk[kv.first] = s->nsrc++;
  // a closure solver adds its terms to the order-N rows through source planes
  if (s->closure)
    for (int k = 0; k < s->nmom; ++k)
      if (s->moms[k].l == s->N) s->qk[k] = s->nsrc++;
  // m ranges of a few indices keep a window within the register and LDS budget
  // of the compiled tiles.  The width is tuned; the program region is sized
  // for the narrowest candidate (most ranges), and program sizes do not depend
  // on the tile.
  if (s->chunk_width <= 0) {
    s->chunk_width = kDefaultChunkWidth;
    if (const char* w = std::getenv("STARMAP_CHUNK_WIDTH")) s->chunk_width = std::max(2, std::atoi(w));
  }
  s->nchunks = sweep_chunk_count(s->N, s->chunk_width);
  for (int p = 0; p < 2; ++p) {
    s->prog_bytes[p] = 0;
    for (int w : kChunkWidths) {
      const SweepProgram pr =
          build_sweep_program(s->N, p, 64, 4, s->dx, s->dy, s->rows, s->dmap, s->qk, sweep_chunk_count(s->N, w));
      s->prog_bytes[p] = std::max(s->prog_bytes[p], program_bytes(pr, s->csize));
    }
    s->prog[p] = build_sweep_program(s->N, p, 64, 4, s->dx, s->dy, s->rows, s->dmap, s->qk, s->nchunks);
    s->prog_bytes[p] = std::max(s->prog_bytes[p], program_bytes(s->prog[p], s->csize));
  }
  s->slots = std::max(s->prog[0].slots, s->prog[1].slots);
  size_t off = 0;
  s->off_state = off;
  // state planes, then the source planes in the storage type (the sweep
  // stages them into LDS like any input plane)
  off += size_t(s->nmom + s->nsrc) * s->plane_bytes_state();
  s->off_src = s->off_state + size_t(s->nmom) * s->plane_bytes_state();
  s->off_decay = off;
  off += size_t(s->dmap.nplanes) * s->plane_bytes_c();
  for (int p = 0; p < 2; ++p) {
    s->off_prog[p] = off;
    off += s->prog_bytes[p];
  }
  s->off_diag = off;
  int max_rows = s->ny + 1;
  s->diag_nblocks = diag_blocks(s->nmom, max_rows, s->diag_rows_per_block);
  off += align256(size_t(s->diag_nblocks) * 4 * 8) + 256 + align256(size_t(s->nmom) * 8);
  if (s->closure) {
    s->off_net = off;
    off += align256(sizeof(ClosureNet));
    // the even sweep's program reading the order-5 moments from the closure planes
    s->off_prog_b = off;
    off += s->prog_bytes[0];
  }
  plan_separable(s);
  if (s->separable) {
    s->off_basis = off;
    off += size_t(s->nbasis) * s->plane_bytes_c();
    s->off_comb = off;
    off += align256(s->comb_tab.size() * 4) + align256(s->comb_cst.size() * 8);
  }
  if (s->has_diffusion) {
    const size_t nd = size_t(s->N + 1);
    s->off_dtmp = off;
    off += nd * s->plane_bytes_state();
    s->off_kappa = off;
    off += nd * s->plane_bytes_c();
    s->off_dtab = off;
    off += align256(nd * 3 * 4);
  }
  if (s->fused) {
    plan_fused(s);
    s->off_state2 = off;
    off += size_t(s->nmom) * s->plane_bytes_state();
    s->off_ftab = off;
    off += align256(s->ftab.size() * 4) + align256(s->fcoef.size() * s->csize);
  }
  s->dev_bytes = off;
}

int upload_one_program(starmap_solver* s, const SweepProgram& pr, size_t region, size_t region_bytes) {
  if (program_bytes(pr, s->csize) > region_bytes) return fail(STARMAP_ENOMEM, "sweep program region too small");
  {
    std::vector<char> buf(region_bytes, 0);
    size_t o = 0;
    {
      std::vector<int32_t> ch;
      for (auto& x : pr.chunks) ch.insert(ch.end(), {x.order0, x.order1, 0, 0});
      std::memcpy(buf.data() + o, ch.data(), ch.size() * 4);
      o += align256(pr.chunks.size() * 16);
    }
    std::vector<int32_t> ords, loads, rws;
    for (auto& x : pr.orders) { ords.insert(ords.end(), {x.load0, x.load1, x.row0, x.row1}); }
    for (auto& x : pr.loads) { loads.insert(loads.end(), {x.k, x.lds, x.ox, x.oy}); }
    for (auto& x : pr.rows) {
      rws.insert(rws.end(), {x.k, x.gslot, x.dk, x.so, x.xo[0], x.xo[1], x.xo[2], x.xo[3], x.yo[0], x.yo[1],
                             x.yo[2], x.yo[3], x.nx, x.ny, 0, 0});
    }
    std::memcpy(buf.data() + o, ords.data(), ords.size() * 4);
    o += align256(pr.orders.size() * 16);
    std::memcpy(buf.data() + o, loads.data(), loads.size() * 4);
    o += align256(pr.loads.size() * 16);
    std::memcpy(buf.data() + o, rws.data(), rws.size() * 4);
    o += align256(pr.rows.size() * 64);
    if (s->csize == 8) {
      std::memcpy(buf.data() + o, pr.coefs.data(), pr.coefs.size() * 8);
    } else {
      std::vector<float> cf(pr.coefs.begin(), pr.coefs.end());
      std::memcpy(buf.data() + o, cf.data(), cf.size() * 4);
    }
    HIP_TRY(hipMemcpyAsync(dptr(s, region), buf.data(), buf.size(), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  return STARMAP_OK;
}

int upload_program(starmap_solver* s) {
  ++s->graph_version;  // tiles, m ranges or LDS size may change: captured launches are stale
  const TileShape ts = sweep_variant(s->variant);
  s->nchunks = sweep_chunk_count(s->N, s->chunk_width);
  for (int p = 0; p < 2; ++p) {
    s->prog[p] = build_sweep_program(s->N, p, ts.tx, ts.ty, s->dx, s->dy, s->rows, s->dmap, s->qk, s->nchunks);
    int rc = upload_one_program(s, s->prog[p], s->off_prog[p], s->prog_bytes[p]);
    if (rc) return rc;
  }
  if (s->closure) {
    // the same even program with the order-5 inputs read from the closure planes
    SweepProgram pb = s->prog[0];
    int a0 = -1, b0 = -1;
    for (int k = 0; k < s->nmom; ++k)
      if (s->moms[k].l == s->N) {
        if (a0 < 0) {
          a0 = k;
          b0 = s->nmom + s->qk[k];
        }
        if (k - a0 != s->nmom + s->qk[k] - b0) return fail(STARMAP_EINVAL, "closure planes are not consecutive");
      }
    for (auto& ld : pb.loads)
      if (ld.k >= a0 && ld.k < a0 + CLOSURE_OUT) ld.k = b0 + (ld.k - a0);
    int rc = upload_one_program(s, pb, s->off_prog_b, s->prog_bytes[0]);
    if (rc) return rc;
  }
  s->slots = std::max(s->prog[0].slots, s->prog[1].slots);
  s->prog_uploaded = true;
  return STARMAP_OK;
}

int ensure_stream(starmap_solver* s) {
  if (!s->bound && !s->stream && !s->owns_stream) {
    HIP_TRY(hipStreamCreate(&s->stream));
    s->owns_stream = true;
  }
  return STARMAP_OK;
}

int upload_materials(starmap_solver* s, double t_eval) {
  // decay planes: c = sigma_a (zeroth moment), sigma_a + sigma_s0 - sigma_sl (l >= 1)
  std::map<int, std::vector<double>> sa, ss;
  auto get = [&](std::map<int, std::vector<double>>& cache, const FieldSource& f, int gx, int gy,
                 std::vector<double>** out) -> int {
    int g = grid_id(gx, gy);
    auto it = cache.find(g);
    if (it == cache.end()) {
      std::vector<double> v;
      int rc = sample(s, f, gx, gy, t_eval, v);
      if (rc) return rc;
      it = cache.emplace(g, std::move(v)).first;
    }
    *out = &it->second;
    return STARMAP_OK;
  };
  for (int p = 0; p < s->dmap.nplanes; ++p) {
    const int gx = s->dmap.plane_gx[p], gy = s->dmap.plane_gy[p], l = s->dmap.plane_l[p];
    std::vector<double>* a = nullptr;
    int rc = get(sa, s->absorption, gx, gy, &a);
    if (rc) return rc;
    std::vector<double> c = *a;
    if (l >= 1) {
      std::vector<double>* b = nullptr;
      rc = get(ss, s->scattering, gx, gy, &b);
      if (rc) return rc;
      for (size_t i = 0; i < c.size(); ++i) c[i] += (*b)[i];
      auto it = s->scattering_order.find(l);
      if (s->anisotropic && it != s->scattering_order.end()) {
        std::vector<double> sl;
        rc = sample(s, it->second, gx, gy, t_eval, sl);
        if (rc) return rc;
        for (size_t i = 0; i < c.size(); ++i) c[i] -= sl[i];
      }
    }
    if (const double d = order_damping(s, l)) for (double& v : c) v += d;
    rc = upload_plane(s, dptr(s, s->off_decay + size_t(p) * s->plane_bytes_c()), gx, gy, c.data(), true);
    if (rc) return rc;
  }
  for (auto& kv : s->source) {
    const int k = kv.first;
    if (s->qk[k] < 0) continue;
    std::vector<double> q;
    int rc = sample(s, kv.second, s->moms[k].gx, s->moms[k].gy, t_eval, q);
    if (rc) return rc;
    rc = upload_plane(s, dptr(s, s->off_src + size_t(s->qk[k]) * s->plane_bytes_state()), s->moms[k].gx,
                      s->moms[k].gy, q.data(), false);
    if (rc) return rc;
  }
  s->materials_ready = true;
  return STARMAP_OK;
}

int load_tune_cache(starmap_solver* s) {
  const char* path = std::getenv("STARMAP_TUNE_CACHE");
  if (!path) return -1;
  std::ifstream f(path);
  std::string line;
  int found = -1;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    int N, nx, ny, st, v, w;
    if (is >> N >> nx >> ny >> st >> v >> w)
      if (N == s->N && nx == s->nx && ny == s->ny && st == s->storage && v >= 0 && v < sweep_variant_count() &&
          w >= 2) {
        found = v;
        s->chunk_width = w;
      }
  }
  return found;
}

int default_variant(const starmap_solver* s) {
  // largest-reuse tile that fits the LDS of one workgroup
  int dev = 0;
  int max_lds = 64 * 1024;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0) max_lds = v;
  }
  for (int v = 0; v < sweep_variant_count(); ++v)
    if (sweep_lds_bytes(v, s->slots, s->storage) <= size_t(max_lds)) return v;
  return -1;
}

static_assert(COMBINE_MAX_TERMS >= STARMAP_MAX_FIELD_TERMS, "combine kernel holds every time factor");

// Basis planes of the separable fields and their combination table.
int upload_basis(starmap_solver* s) {
  for (int b = 0; b < s->nbasis; ++b) {
    const auto& bs = s->basis[size_t(b)];
    std::vector<double> v;
    int rc = sample_basis(s, *bs.field, bs.term, bs.gx, bs.gy, v);
    if (rc) return rc;
    rc = upload_plane(s, dptr(s, s->off_basis + size_t(b) * s->plane_bytes_c()), bs.gx, bs.gy, v.data(), true);
    if (rc) return rc;
  }
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_comb), s->comb_tab.data(), s->comb_tab.size() * 4, hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_comb + align256(s->comb_tab.size() * 4)), s->comb_cst.data(),
                         s->comb_cst.size() * 8, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->basis_ready = true;
  s->static_done = false;
  return STARMAP_OK;
}

// Decay and source planes at time t_eval from the separable fields, on the
// device: the first call forms every plane, later calls only those with a
// time factor.  The time factors travel as kernel arguments.
int combine_materials(starmap_solver* s, double t_eval) {
  if (!s->basis_ready) {
    int rc = upload_basis(s);
    if (rc) return rc;
  }
  CombineArgs c{};
  for (size_t i = 0; i < s->time_terms.size(); ++i) {
    c.a[i] = s->time_terms[i].time(s->time_terms[i].time_ctx, t_eval);
    if (!std::isfinite(c.a[i])) return fail(STARMAP_EINVAL, "time factor is not finite");
  }
  const int32_t* tab = reinterpret_cast<const int32_t*>(dptr(s, s->off_comb));
  c.basis = dptr(s, s->off_basis);
  c.first = tab + s->tab_first;
  c.entries = tab + s->tab_entries;
  c.cst = reinterpret_cast<const double*>(dptr(s, s->off_comb + align256(s->comb_tab.size() * 4)));
  c.plane_stride = s->plane_stride;
  const int w = s->static_done ? 1 : 0;
  if (s->nlist[w]) {  // decay planes, compute type
    c.out = dptr(s, s->off_decay);
    c.list = tab + s->tab_list[w];
    c.nlist = s->nlist[w];
    HIP_TRY(launch_combine(s->storage, true, c, s->stream));
  }
  if (s->nlist[2 + w]) {  // source planes, storage type
    c.out = dptr(s, s->off_src);
    c.list = tab + s->tab_list[2 + w];
    c.nlist = s->nlist[2 + w];
    HIP_TRY(launch_combine(s->storage, false, c, s->stream));
  }
  s->static_done = true;
  s->materials_ready = true;
  return STARMAP_OK;
}

// Materials for a time-independent or separable problem at t_eval.
int ensure_materials(starmap_solver* s, double t_eval) {
  if (s->separable && !s->time_dependent) return combine_materials(s, t_eval);
  return upload_materials(s, t_eval);
}

// D_N: kappa on the grid of every order-N moment (compute type), the plane
// table, and the stability check of the explicit diffusion step.
int upload_diffusion(starmap_solver* s) {
  std::vector<int32_t> tab;
  const double lim = s->dt * (2.0 / (s->dx * s->dx) + 2.0 / (s->dy * s->dy));
  int j = 0;
  for (int k = 0; k < s->nmom; ++k) {
    if (s->moms[k].l != s->N) continue;
    const int gx = s->moms[k].gx, gy = s->moms[k].gy;
    std::vector<double> v;
    int rc = sample(s, s->diffusion, gx, gy, 0.0, v);
    if (rc) return rc;
    for (double x : v) {
      if (!(x >= 0.0) || !std::isfinite(x)) return fail(STARMAP_EINVAL, "diffusion coefficient must be finite and >= 0");
      if (x * lim > 1.0) return fail(STARMAP_EINVAL, "diffusion step unstable: kappa dt (2/dx^2 + 2/dy^2) > 1");
    }
    rc = upload_plane(s, dptr(s, s->off_kappa + size_t(j) * s->plane_bytes_c()), gx, gy, v.data(), true);
    if (rc) return rc;
    tab.insert(tab.end(), {k, gx, gy});
    ++j;
  }
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_dtab), tab.data(), tab.size() * 4, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->diffusion_ready = true;
  return STARMAP_OK;
}

// D_tau on the order-N moments.
int diffuse(starmap_solver* s, double tau) {
  DiffusionArgs a;
  a.u = dptr(s, s->off_state);
  a.tmp = dptr(s, s->off_dtmp);
  a.kappa = dptr(s, s->off_kappa);
  a.tab = reinterpret_cast<const int*>(dptr(s, s->off_dtab));
  a.plane_stride = s->plane_stride;
  a.pitch = s->pitch;
  a.nx = s->nx;
  a.ny = s->ny;
  a.px = s->px;
  a.py = s->py;
  a.nplanes = s->N + 1;
  a.rdx2 = 1.0 / (s->dx * s->dx);
  a.rdy2 = 1.0 / (s->dy * s->dy);
  a.tau = tau;
  HIP_TRY(launch_diffusion(s->storage, a, (s->nx + 1) * (s->ny + 1), s->stream));
  return STARMAP_OK;
}

// initial state planes (zero where no initial field is set)
int upload_initial(starmap_solver* s) {
  HIP_TRY(hipMemsetAsync(dptr(s, s->off_state), 0, size_t(s->nmom) * s->plane_bytes_state(), s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int k = 0; k < s->nmom; ++k) {
    auto it = s->initial.find(k);
    if (it == s->initial.end() || !it->second.set()) continue;
    std::vector<double> v;
    int rc = sample(s, it->second, s->moms[k].gx, s->moms[k].gy, 0.0, v);
    if (rc) return rc;
    rc = upload_plane(s, dptr(s, s->off_state + size_t(k) * s->plane_bytes_state()), s->moms[k].gx,
                      s->moms[k].gy, v.data(), false);
    if (rc) return rc;
  }
  return STARMAP_OK;
}

int ensure_device(starmap_solver* s) {
  if (s->device_ready) return STARMAP_OK;
  // decay planes may have been added (anisotropic scattering, filter damping)
  // after the fused mode was chosen
  if (s->fused && fused_lds_bytes(s->storage, s->nmom, s->dmap.nplanes) > size_t(max_lds_bytes()))
    return fail(STARMAP_EINVAL, "parity-fused tile (moments and decay planes) does not fit the LDS");
  int rc = ensure_stream(s);
  if (rc) return rc;
  if (!s->dev) {
    HIP_TRY(hipMalloc(&s->dev, s->dev_bytes));
    s->owns_dev = true;
  }
  // zero everything once (padding included), then the initial state
  HIP_TRY(hipMemsetAsync(s->dev, 0, s->dev_bytes, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  rc = upload_initial(s);
  if (rc) return rc;
  if (s->has_diffusion) {
    rc = upload_diffusion(s);
    if (rc) return rc;
  }
  // diagnostics geometry: valid points per plane
  {
    std::vector<int32_t> geo(size_t(s->nmom) * 2);
    for (int k = 0; k < s->nmom; ++k) {
      geo[k] = points_x(s, s->moms[k].gx);
      geo[s->nmom + k] = points_y(s, s->moms[k].gy);
    }
    size_t off = s->off_diag + align256(size_t(s->diag_nblocks) * 4 * 8) + 256;
    HIP_TRY(hipMemcpyAsync(dptr(s, off), geo.data(), geo.size() * 4, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
  }
  if (s->variant < 0) {
    int v = load_tune_cache(s);
    if (v < 0) v = default_variant(s);
    if (v < 0) return fail(STARMAP_ENOMEM, "no sweep tile fits the LDS for this moment order");
    s->variant = v;
  }
  rc = upload_program(s);
  if (rc) return rc;
  s->device_ready = true;
  return STARMAP_OK;
}

template <typename C>
int launch_one(starmap_solver* s, int parity, double tau) {
  SweepArgs<C> a;
  const auto& pr = s->prog[parity];
  // a fused closure solver's even sweep reads the order-5 moments where the
  // last odd sweep wrote them
  const bool from_b = parity == 0 && s->closure && s->closure_fused && s->c5_flip;
  char* base = dptr(s, from_b ? s->off_prog_b : s->off_prog[parity]);
  size_t o = 0;
  a.chunks = reinterpret_cast<const int4*>(base + o);
  o += align256(pr.chunks.size() * 16);
  a.orders = reinterpret_cast<const int4*>(base + o);
  o += align256(pr.orders.size() * 16);
  a.loads = reinterpret_cast<const int4*>(base + o);
  o += align256(pr.loads.size() * 16);
  a.rows = reinterpret_cast<const int*>(base + o);
  o += align256(pr.rows.size() * 64);
  a.rcoef = reinterpret_cast<const C*>(base + o);
  a.u = dptr(s, s->off_state);
  a.decay = reinterpret_cast<const C*>(dptr(s, s->off_decay));
  a.plane_stride = s->plane_stride;
  a.pitch = s->pitch;
  a.nx = s->nx;
  a.ny = s->ny;
  a.px = s->px;
  a.py = s->py;
  const TileShape ts = sweep_variant(s->variant);
  a.ntx = (s->nx + 1 + ts.tx - 1) / ts.tx;
  a.nty = (s->ny + 1 + ts.ty - 1) / ts.ty;
  a.nchunks = int(pr.chunks.size());
  a.zero_off = pr.zero_off;
  a.parity = parity;
  a.strip = s->tile_strip;
  a.tau = C(tau);
  HIP_TRY(launch_sweep(s->storage, s->variant, &a, s->slots, s->stream));
  return STARMAP_OK;
}

double sweep_bytes_of(const starmap_solver* s, int parity);

int sweep(starmap_solver* s, int parity, double tau, bool with_closure = true) {
  const bool fused_closure = parity == 1 && s->closure && with_closure && s->closure_fused;
  if (parity == 1 && s->closure && with_closure && !s->closure_fused) {
    int rc = closure_before_odd(s);
    if (rc) return rc;
  }
  if (s->profiling) {
    if (s->ev_used + 2 > s->ev.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        s->ev.push_back(e);
      }
    }
    HIP_TRY(hipEventRecord(s->ev[s->ev_used], s->stream));
  }
  int rc = fused_closure ? closure_odd_sweep(s, tau)
           : s->storage == STORE_FP64 ? launch_one<double>(s, parity, tau) : launch_one<float>(s, parity, tau);
  if (rc) return rc;
  if (s->profiling) {
    HIP_TRY(hipEventRecord(s->ev[s->ev_used + 1], s->stream));
    s->ev_used += 2;
    if (s->sweep_bytes_cache[parity] < 0) s->sweep_bytes_cache[parity] = sweep_bytes_of(s, parity);
    s->prof_bytes += s->sweep_bytes_cache[parity];
  }
  return STARMAP_OK;
}

// The even part of a step: S^e_tau, or S^e_{tau/2} D_tau S^e_{tau/2} with the
// D_N diffusion step.
int even_part(starmap_solver* s, double tau) {
  if (!s->has_diffusion) return sweep(s, 0, tau);
  int r = sweep(s, 0, 0.5 * tau);
  if (!r) r = diffuse(s, tau);
  if (!r) r = sweep(s, 0, 0.5 * tau);
  return r;
}

void drop_pair_graphs(starmap_solver* s) {
  for (auto& kv : s->pair_graphs) (void)hipGraphExecDestroy(kv.second);
  s->pair_graphs.clear();
}

constexpr int kMaxGraphPairs = 16;

// pairs times (S^e_dt, S^o_dt), as launches of captured graphs of 16, 8, 4,
// 2 and 1 pairs (each captured on first use from the same calls the eager
// path makes, so the kernels and their arguments are the same).
int run_pairs_graphed(starmap_solver* s, int64_t pairs, double dt) {
  if (s->pair_graphs_version != s->graph_version) {
    drop_pair_graphs(s);
    s->pair_graphs_version = s->graph_version;
  }
  while (pairs > 0) {
    int p = kMaxGraphPairs;
    while (p > pairs) p >>= 1;
    // a fused closure solver's launches also depend on where the order-5
    // moments sit (each odd sweep moves them)
    const int key = 2 * p + s->c5_flip;
    auto it = s->pair_graphs.find(key);
    const bool cached = it != s->pair_graphs.end();
    if (!cached) {
      HIP_TRY(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
      int rc = STARMAP_OK;
      for (int i = 0; i < p && !rc; ++i) {
        rc = even_part(s, dt);
        if (!rc) rc = sweep(s, 1, dt);
      }
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(s->stream, &g);
      if (rc || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc) return rc;
        HIP_TRY(e);
      }
      hipGraphExec_t x = nullptr;
      const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIP_TRY(ei);
      it = s->pair_graphs.emplace(key, x).first;
    }
    HIP_TRY(hipGraphLaunch(it->second, s->stream));
    // the capture moved the host-side order-5 location already; a replay does it here
    if (cached && s->closure && s->closure_fused) s->c5_flip ^= (p & 1);
    pairs -= p;
  }
  return STARMAP_OK;
}

int validate(const starmap_problem* p) {
  if (!p) return fail(STARMAP_EINVAL, "problem is NULL");
  if (p->N < 1 || p->N > 99) return fail(STARMAP_EINVAL, "moment order N must be in 1..99");
  if (p->n[0] < 2 || p->n[1] < 2) return fail(STARMAP_EINVAL, "need at least 2 cells per axis");
  if (int64_t(p->n[0]) * p->n[1] > (int64_t(1) << 30)) return fail(STARMAP_EINVAL, "grid too large");
  for (int a = 0; a < 2; ++a)
    if (p->bc[a] != STARMAP_BC_PERIODIC && p->bc[a] != STARMAP_BC_EXTRAPOLATION)
      return fail(STARMAP_EINVAL, "unknown boundary type");
  if (!(p->ax[1] > p->ax[0]) || !(p->ax[3] > p->ax[2])) return fail(STARMAP_EINVAL, "empty domain");
  if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return fail(STARMAP_EINVAL, "cfl must be positive");
  if (!(p->t_final > 0.0) || !std::isfinite(p->t_final)) return fail(STARMAP_EINVAL, "t_final must be positive");
  if (p->precision < STARMAP_FP64 || p->precision > STARMAP_BF16) return fail(STARMAP_EINVAL, "unknown precision");
  if (p->closure != STARMAP_CLOSURE_PN && p->closure != STARMAP_CLOSURE_LEARNED)
    return fail(STARMAP_EINVAL, "unknown closure");
  return STARMAP_OK;
}

int check_k(const starmap_solver* s, int k) {
  if (k < 0 || k >= s->nmom) return fail(STARMAP_EINVAL, "moment index out of range");
  return STARMAP_OK;
}

// A field is about to change: a field with separable terms is fixed once the
// device plan exists; any other change re-samples the basis planes.
int field_change(starmap_solver* s, const FieldSource& f) {
  if (s->device_ready && s->separable && !f.terms.empty())
    return fail(STARMAP_ESTATE, "a field given by separable terms is fixed after the first device call");
  s->basis_ready = false;
  return STARMAP_OK;
}

int set_field(starmap_solver* s, FieldSource& f, starmap_field_fn fn, void* ctx, int td) {
  int rc = field_change(s, f);
  if (rc) return rc;
  f.fn = fn;
  f.ctx = ctx;
  f.time_dependent = td != 0;
  f.terms.clear();
  for (int g = 0; g < 4; ++g) f.has_array[g] = false;
  if (td) s->time_dependent = true;
  s->materials_ready = false;
  return STARMAP_OK;
}

}  // namespace detail
}  // namespace starmap

// ===================================================================== ABI
extern "C" {

int starmap_num_moments(int32_t N) {
  if (N < 0 || N > 99) return fail(STARMAP_EINVAL, "moment order out of range");
  return moment_count(N);
}

int starmap_moment_info(int32_t N, int32_t k, int32_t* is_imag, int32_t* l, int32_t* m, int32_t* gx,
                        int32_t* gy) {
  if (N < 0 || N > 99) return fail(STARMAP_EINVAL, "moment order out of range");
  const auto moms = moment_list(N);
  if (k < 0 || k >= int(moms.size())) return fail(STARMAP_EINVAL, "moment index out of range");
  if (is_imag) *is_imag = moms[k].imag;
  if (l) *l = moms[k].l;
  if (m) *m = moms[k].m;
  if (gx) *gx = moms[k].gx;
  if (gy) *gy = moms[k].gy;
  return STARMAP_OK;
}

int starmap_closure_pn(int32_t N, int32_t axis, int32_t* cols, double* vals) {
  if (N < 0 || N > 99) return fail(STARMAP_EINVAL, "moment order out of range");
  if ((axis != 0 && axis != 1) || !cols || !vals) return fail(STARMAP_EINVAL, "bad arguments");
  try {
    const auto rows = closure_pn(N);
    for (size_t k = 0; k < rows.size(); ++k) {
      const int n = axis == 0 ? rows[k].nx : rows[k].ny;
      const Coupling* c = axis == 0 ? rows[k].x : rows[k].y;
      for (int t = 0; t < 4; ++t) {
        cols[4 * k + t] = t < n ? c[t].col : -1;
        vals[4 * k + t] = t < n ? c[t].val : 0.0;
      }
    }
  } catch (const std::exception& e) {
    return fail(STARMAP_EINVAL, e.what());
  }
  return STARMAP_OK;
}

int starmap_plan_check(int32_t N, int32_t tile_x, int32_t tile_y, int32_t nchunks) {
  if (N < 1 || N > 99 || tile_x < 1 || tile_y < 1 || nchunks < 1) return fail(STARMAP_EINVAL, "bad arguments");
  try {
    const auto rows = closure_pn(N);
    const DecayMap dm = decay_map(N, true);
    std::vector<int32_t> qk(moment_count(N), -1);
    qk[0] = 0;  // isotropic source on the zeroth moment
    if (moment_count(N) > 3) qk[3] = 1;  // and one on an even moment of order 2
    if (moment_count(N) > 1) qk[1] = 2;  // and one on an odd moment
    // and a beam: sources on every moment
    std::vector<int32_t> all(moment_count(N));
    for (int k = 0; k < moment_count(N); ++k) all[k] = k;
    for (const auto* q : {&qk, &all})
      for (int p = 0; p < 2; ++p) {
        const SweepProgram pr = build_sweep_program(N, p, tile_x, tile_y, 0.1, 0.2, rows, dm, *q, nchunks);
        const std::string e = validate_sweep_program(N, pr, rows, *q);
        if (!e.empty()) return fail(STARMAP_EINVAL, "sweep program check failed: " + e);
      }
  } catch (const std::exception& e) {
    return fail(STARMAP_EINVAL, e.what());
  }
  return STARMAP_OK;
}

int starmap_direction_moments(int32_t N, double ox, double oy, double oz, double* out) {
  if (N < 0 || N > 99 || !out) return fail(STARMAP_EINVAL, "bad arguments");
  const double n2 = ox * ox + oy * oy + oz * oz;
  if (!(std::fabs(n2 - 1.0) < 1e-9)) return fail(STARMAP_EINVAL, "direction must be a unit vector");
  const std::vector<double> v = direction_moments(N, ox, oy, oz);
  std::copy(v.begin(), v.end(), out);
  return STARMAP_OK;
}

int starmap_spectral_radius(int32_t N, double* rho) {
  if (N < 0 || N > 99 || !rho) return fail(STARMAP_EINVAL, "bad arguments");
  *rho = spectral_radius_x(closure_pn(N));
  return STARMAP_OK;
}

int starmap_create(const starmap_problem* prob, starmap_solver** out) {
  if (!out) return fail(STARMAP_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(prob);
  if (rc) return rc;
  std::unique_ptr<starmap_solver> s(new (std::nothrow) starmap_solver());
  if (!s) return fail(STARMAP_ENOMEM, "out of host memory");
  s->prob = *prob;
  s->N = prob->N;
  s->closure = prob->closure == STARMAP_CLOSURE_LEARNED;
  if (s->closure && s->N != 5) return fail(STARMAP_EINVAL, "the learned closure is defined for N = 5");
  s->nmom = moment_count(s->N);
  try {
    s->moms = moment_list(s->N);
    s->rows = closure_pn(s->N);
  } catch (const std::exception& e) {
    return fail(STARMAP_EINVAL, e.what());
  }
  s->nx = prob->n[0];
  s->ny = prob->n[1];
  s->px = prob->bc[0] == STARMAP_BC_PERIODIC ? 1 : 0;
  s->py = prob->bc[1] == STARMAP_BC_PERIODIC ? 1 : 0;
  s->dx = (prob->ax[1] - prob->ax[0]) / s->nx;
  s->dy = (prob->ax[3] - prob->ax[2]) / s->ny;
  s->rho = spectral_radius_x(s->rows);
  time_step(prob->cfl, s->dx, s->dy, s->rho, prob->t_final, &s->dt, &s->steps_total);
  s->storage = prob->precision == STARMAP_FP64 ? STORE_FP64 : prob->precision == STARMAP_FP32 ? STORE_FP32 : STORE_BF16;
  s->ssize = s->storage == STORE_FP64 ? 8 : s->storage == STORE_FP32 ? 4 : 2;
  s->csize = s->storage == STORE_FP64 ? 8 : 4;
  s->pitch = int((s->nx + 1 + 63) / 64 * 64);
  s->nrows = s->ny + 1;
  s->plane_stride = (int64_t(s->pitch) * s->nrows + 127) / 128 * 128;
  if (const char* e = std::getenv("STARMAP_TILE_STRIP")) {
    const int v = std::atoi(e);
    s->tile_strip = (v >= 2 || v <= -2) ? v : 1;
  }
  // The kernels address a plane with 32-bit byte offsets (element offset
  // times the storage or compute size, whichever is larger): keep every such
  // offset below 2^31.
  if (s->plane_stride * int64_t(std::max(s->ssize, s->csize)) >= (int64_t(1) << 31))
    return fail(STARMAP_EINVAL, "grid too large for 32-bit plane byte offsets");
  layout(s.get());
  *out = s.release();
  return STARMAP_OK;
}

void starmap_destroy(starmap_solver* s) {
  if (!s) return;
  if (s->device_ready) (void)hipStreamSynchronize(s->stream);
  drop_pair_graphs(s);
  if (s->sample_buf) (void)hipFree(s->sample_buf);
  if (s->owns_dev && s->dev) (void)hipFree(s->dev);
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  if (s->owns_stream && s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

int starmap_set_absorption(starmap_solver* s, starmap_field_fn f, void* ctx, int32_t td) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  return set_field(s, s->absorption, f, ctx, td);
}

int starmap_set_scattering(starmap_solver* s, starmap_field_fn f, void* ctx, int32_t td) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  return set_field(s, s->scattering, f, ctx, td);
}

int starmap_set_scattering_order(starmap_solver* s, int32_t l, starmap_field_fn f, void* ctx, int32_t td) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (l < 1 || l > s->N) return fail(STARMAP_EINVAL, "order must be in 1..N");
  if (s->device_ready && !s->anisotropic)
    return fail(STARMAP_ESTATE, "anisotropic scattering must be set before the first device call");
  s->anisotropic = true;
  int rc = set_field(s, s->scattering_order[l], f, ctx, td);
  if (rc) return rc;
  if (!s->device_ready) layout(s);
  return STARMAP_OK;
}

int starmap_set_source(starmap_solver* s, int32_t k, starmap_field_fn f, void* ctx, int32_t td) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  int rc = check_k(s, k);
  if (rc) return rc;
  if (s->closure && s->moms[k].l == s->N)
    return fail(STARMAP_EINVAL, "a closure solver carries its own terms on the order-N moments; no source there");
  const bool is_new = s->source.find(k) == s->source.end() || !s->source[k].set();
  if (s->device_ready && is_new) return fail(STARMAP_ESTATE, "new source moments must be set before the first device call");
  rc = set_field(s, s->source[k], f, ctx, td);
  if (rc) return rc;
  if (!s->device_ready) layout(s);
  return STARMAP_OK;
}

int starmap_add_field_term(starmap_solver* s, int32_t which, int32_t index, starmap_field_fn space,
                           void* space_ctx, starmap_time_fn time, void* time_ctx) {
  if (!s || !space || !time) return fail(STARMAP_EINVAL, "bad arguments");
  if (s->device_ready) return fail(STARMAP_ESTATE, "field terms must be added before the first device call");
  FieldSource* f = nullptr;
  switch (which) {
    case STARMAP_FIELD_ABSORPTION: f = &s->absorption; break;
    case STARMAP_FIELD_SCATTERING: f = &s->scattering; break;
    case STARMAP_FIELD_SCATTERING_ORDER:
      if (index < 1 || index > s->N) return fail(STARMAP_EINVAL, "order must be in 1..N");
      s->anisotropic = true;
      f = &s->scattering_order[index];
      break;
    case STARMAP_FIELD_SOURCE: {
      int rc = check_k(s, index);
      if (rc) return rc;
      if (s->closure && s->moms[index].l == s->N)
        return fail(STARMAP_EINVAL, "a closure solver carries its own terms on the order-N moments; no source there");
      f = &s->source[index];
      break;
    }
    default: return fail(STARMAP_EINVAL, "unknown field selector for a separable term");
  }
  if (f->terms.empty()) {  // a term replaces a callback or arrays
    f->fn = nullptr;
    f->ctx = nullptr;
    f->time_dependent = false;
    for (int g = 0; g < 4; ++g) f->has_array[g] = false;
  }
  f->terms.push_back({space, space_ctx, time, time_ctx});
  s->materials_ready = false;
  layout(s);
  if (s->time_terms.size() > size_t(STARMAP_MAX_FIELD_TERMS)) {
    f->terms.pop_back();
    layout(s);
    return fail(STARMAP_EINVAL, "too many separable field terms");
  }
  return STARMAP_OK;
}

int starmap_set_filter_damping(starmap_solver* s, const double* damping) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (damping) {
    for (int l = 0; l <= s->N; ++l)
      if (!(damping[l] >= 0.0) || !std::isfinite(damping[l]))
        return fail(STARMAP_EINVAL, "filter damping must be finite and >= 0");
    if (s->device_ready && !s->anisotropic)
      return fail(STARMAP_ESTATE, "filter damping must first be set before the first device call");
    s->damping.assign(damping, damping + s->N + 1);
  } else {
    s->damping.clear();
  }
  if (!s->device_ready) {
    if (damping) s->anisotropic = true;  // per-order decay planes
    layout(s);
  } else if (s->separable) {
    // the decay outputs come first in the combination table, in plane order
    for (int p = 0; p < s->dmap.nplanes; ++p) s->comb_cst[size_t(p)] = order_damping(s, s->dmap.plane_l[p]);
    s->basis_ready = false;
  }
  s->materials_ready = false;
  return STARMAP_OK;
}

int starmap_set_fused(starmap_solver* s, int32_t enable) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (s->device_ready) return fail(STARMAP_ESTATE, "the fused mode must be chosen before the first device call");
  if (enable && s->N > STARMAP_FUSED_MAX_ORDER)
    return fail(STARMAP_EINVAL, "parity-fused passes hold all moments of a tile in LDS: order too high");
  if (enable && s->closure) return fail(STARMAP_EINVAL, "parity-fused passes do not take the learned closure");
  if (enable && fused_lds_bytes(s->storage, s->nmom, s->dmap.nplanes) > size_t(max_lds_bytes()))
    return fail(STARMAP_EINVAL, "parity-fused tile (moments and decay planes) does not fit the LDS");
  s->fused = enable != 0;
  layout(s);
  return STARMAP_OK;
}

int starmap_set_diffusion(starmap_solver* s, starmap_field_fn kappa, void* ctx) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (s->device_ready) return fail(STARMAP_ESTATE, "the D_N diffusion must be set before the first device call");
  if (kappa && s->closure) return fail(STARMAP_EINVAL, "the learned closure and D_N do not combine");
  s->diffusion = FieldSource{};
  s->diffusion.fn = kappa;
  s->diffusion.ctx = ctx;
  s->has_diffusion = kappa != nullptr;
  layout(s);
  return STARMAP_OK;
}

int starmap_set_initial(starmap_solver* s, int32_t k, starmap_field_fn f, void* ctx) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  int rc = check_k(s, k);
  if (rc) return rc;
  if (s->device_ready) return fail(STARMAP_ESTATE, "initial values must be set before the first device call");
  FieldSource& fs = s->initial[k];
  fs.fn = f;
  fs.ctx = ctx;
  return STARMAP_OK;
}

int starmap_set_field_array(starmap_solver* s, int32_t which, int32_t k, const double* vals) {
  if (!s || !vals) return fail(STARMAP_EINVAL, "bad arguments");
  int rc = check_k(s, k);
  if (rc) return rc;
  const int gx = s->moms[k].gx, gy = s->moms[k].gy, g = grid_id(gx, gy);
  const size_t n = size_t(points_x(s, gx)) * points_y(s, gy);
  FieldSource* f = nullptr;
  switch (which) {
    case STARMAP_FIELD_ABSORPTION: f = &s->absorption; break;
    case STARMAP_FIELD_SCATTERING: f = &s->scattering; break;
    case STARMAP_FIELD_SOURCE: {
      if (s->closure && s->moms[k].l == s->N)
        return fail(STARMAP_EINVAL, "a closure solver carries its own terms on the order-N moments; no source there");
      const bool is_new = s->source.find(k) == s->source.end() || !s->source[k].set();
      if (s->device_ready && is_new) return fail(STARMAP_ESTATE, "new source moments must be set before the first device call");
      f = &s->source[k];
      break;
    }
    case STARMAP_FIELD_INITIAL:
      if (s->device_ready) return fail(STARMAP_ESTATE, "initial values must be set before the first device call");
      f = &s->initial[k];
      break;
    default: return fail(STARMAP_EINVAL, "unknown field selector");
  }
  if (which != STARMAP_FIELD_INITIAL) {
    rc = field_change(s, *f);
    if (rc) return rc;
  }
  f->arrays[g].assign(vals, vals + n);
  f->has_array[g] = true;
  f->terms.clear();
  if (which != STARMAP_FIELD_INITIAL) {
    s->materials_ready = false;
    if (!s->device_ready) layout(s);
  }
  return STARMAP_OK;
}

int starmap_moment_shape(const starmap_solver* s, int32_t k, int32_t* nx_k, int32_t* ny_k, double* x0_k,
                         double* y0_k) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  int rc = check_k(s, k);
  if (rc) return rc;
  const int gx = s->moms[k].gx, gy = s->moms[k].gy;
  if (nx_k) *nx_k = points_x(s, gx);
  if (ny_k) *ny_k = points_y(s, gy);
  if (x0_k) *x0_k = gx == AXIS_CELL ? s->prob.ax[0] + 0.5 * s->dx : s->prob.ax[0] + s->px * s->dx;
  if (y0_k) *y0_k = gy == AXIS_CELL ? s->prob.ax[2] + 0.5 * s->dy : s->prob.ax[2] + s->py * s->dy;
  return STARMAP_OK;
}

int starmap_time(const starmap_solver* s, double* t, double* dt, int64_t* done, int64_t* total) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (t) *t = s->t;
  if (dt) *dt = s->dt;
  if (done) *done = s->steps_done;
  if (total) *total = s->steps_total;
  return STARMAP_OK;
}

int starmap_workspace_bytes(const starmap_solver* s, size_t* bytes) {
  if (!s || !bytes) return fail(STARMAP_EINVAL, "bad arguments");
  *bytes = s->dev_bytes;
  return STARMAP_OK;
}

int starmap_bind_device(starmap_solver* s, void* dev_ptr, size_t bytes, void* hip_stream) {
  if (!s || !dev_ptr) return fail(STARMAP_EINVAL, "bad arguments");
  if (s->device_ready || s->dev) return fail(STARMAP_ESTATE, "device memory already in use");
  if (bytes < s->dev_bytes) return fail(STARMAP_ENOMEM, "bound workspace is smaller than starmap_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(dev_ptr) % 256) return fail(STARMAP_EINVAL, "workspace must be 256-byte aligned");
  s->dev = dev_ptr;
  s->owns_dev = false;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->bound = true;
  return STARMAP_OK;
}

int starmap_advance(starmap_solver* s, int64_t nsteps) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (nsteps < 0) return fail(STARMAP_EINVAL, "negative step count");
  if (nsteps == 0) return STARMAP_OK;
  if (s->closure && (s->time_dependent || s->separable))
    return fail(STARMAP_EINVAL, "the learned closure needs time-independent data");
  if (s->closure && s->has_diffusion) return fail(STARMAP_EINVAL, "the learned closure and D_N do not combine");
  int rc = ensure_device(s);
  if (rc) return rc;
  const double dt = s->dt;
  auto even = [&]() -> int { return even_part(s, dt); };
  if (!s->time_dependent && !s->separable && s->fused && !s->has_diffusion) {
    // pairs (S^o, S^e) in one pass each, ping-ponging between two state
    // buffers, then the closing odd half-step
    if (!s->materials_ready) {
      rc = upload_materials(s, s->t + 0.5 * dt);
      if (rc) return rc;
    }
    size_t cur = s->off_state, other = s->off_state2;
    for (int64_t i = 0; i < nsteps; ++i) {
      rc = fused_pass(s, cur, other, i == 0 ? 0.5 * dt : dt, dt);
      if (rc) return rc;
      std::swap(cur, other);
    }
    if (cur != s->off_state)
      HIP_TRY(hipMemcpyAsync(dptr(s, s->off_state), dptr(s, cur), size_t(s->nmom) * s->plane_bytes_state(),
                             hipMemcpyDeviceToDevice, s->stream));
    rc = sweep(s, 1, 0.5 * dt);
    if (rc) return rc;
  } else if (!s->time_dependent && !s->separable) {
    if (!s->materials_ready) {
      rc = upload_materials(s, s->t + 0.5 * dt);
      if (rc) return rc;
    }
    rc = sweep(s, 1, 0.5 * dt);
    if (rc) return rc;
    // nsteps - 1 pairs (S^e_dt, S^o_dt), then S^e_dt, S^o_{dt/2}; the pairs
    // replay captured graphs unless launches are being timed one by one (or
    // the stream is the null stream, which cannot be captured)
    const int64_t pairs = nsteps - 1;
    if (pairs > 0 && s->use_graphs && !s->profiling && s->stream) {
      rc = run_pairs_graphed(s, pairs, dt);
      if (rc) return rc;
    } else {
      for (int64_t i = 0; i < pairs; ++i) {
        rc = even();
        if (!rc) rc = sweep(s, 1, dt);
        if (rc) return rc;
      }
    }
    rc = even();
    if (!rc) rc = sweep(s, 1, 0.5 * dt);
    if (rc) return rc;
  } else if (s->separable && !s->time_dependent) {
    // time-separable data: decay and source planes formed on the device per step
    for (int64_t i = 0; i < nsteps; ++i) {
      rc = combine_materials(s, (s->steps_done + i) * dt + 0.5 * dt);
      if (rc) return rc;
      rc = sweep(s, 1, 0.5 * dt);
      if (rc) return rc;
      rc = even();
      if (rc) return rc;
      rc = sweep(s, 1, 0.5 * dt);
      if (rc) return rc;
    }
  } else {
    for (int64_t i = 0; i < nsteps; ++i) {
      HIP_TRY(hipStreamSynchronize(s->stream));
      rc = upload_materials(s, (s->steps_done + i) * dt + 0.5 * dt);
      if (rc) return rc;
      rc = sweep(s, 1, 0.5 * dt);
      if (rc) return rc;
      rc = even();
      if (rc) return rc;
      rc = sweep(s, 1, 0.5 * dt);
      if (rc) return rc;
    }
  }
  if (s->closure) {
    rc = closure_settle(s);
    if (rc) return rc;
  }
  s->steps_done += nsteps;
  s->t = double(s->steps_done) * dt;
  return STARMAP_OK;
}

int starmap_run(starmap_solver* s) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  int rc = starmap_advance(s, s->steps_total - s->steps_done);
  if (rc) return rc;
  return starmap_synchronize(s);
}

int starmap_sweep(starmap_solver* s, int32_t parity, double tau, int32_t nsweeps) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if ((parity != 0 && parity != 1) || nsweeps < 0 || !std::isfinite(tau)) return fail(STARMAP_EINVAL, "bad arguments");
  int rc = ensure_device(s);
  if (rc) return rc;
  if (!s->materials_ready) {
    rc = ensure_materials(s, s->t + 0.5 * s->dt);
    if (rc) return rc;
  }
  for (int i = 0; i < nsweeps; ++i) {
    rc = sweep(s, parity, tau);
    if (rc) return rc;
  }
  if (s->closure) return closure_settle(s);
  return STARMAP_OK;
}

int starmap_synchronize(starmap_solver* s) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (!s->device_ready) return STARMAP_OK;
  HIP_TRY(hipStreamSynchronize(s->stream));
  return STARMAP_OK;
}

int starmap_get_moment(const starmap_solver* cs, int32_t k, double* out) {
  starmap_solver* s = const_cast<starmap_solver*>(cs);
  if (!s || !out) return fail(STARMAP_EINVAL, "bad arguments");
  int rc = check_k(s, k);
  if (rc) return rc;
  rc = ensure_device(s);
  if (rc) return rc;
  const size_t n = size_t(s->plane_stride);
  const char* src = dptr(s, s->off_state + size_t(k) * s->plane_bytes_state());
  const int gx = s->moms[k].gx, gy = s->moms[k].gy;
  if (s->storage == STORE_FP64) {
    std::vector<double> buf(n);
    HIP_TRY(hipMemcpyAsync(buf.data(), src, n * 8, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    gather_plane(s, gx, gy, buf.data(), out);
  } else if (s->storage == STORE_FP32) {
    std::vector<float> buf(n);
    HIP_TRY(hipMemcpyAsync(buf.data(), src, n * 4, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    gather_plane(s, gx, gy, buf.data(), out);
  } else {
    std::vector<uint16_t> buf(n);
    HIP_TRY(hipMemcpyAsync(buf.data(), src, n * 2, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    gather_plane(s, gx, gy, buf.data(), out);
  }
  return STARMAP_OK;
}

int starmap_state_bytes(const starmap_solver* s, size_t* bytes) {
  if (!s || !bytes) return fail(STARMAP_EINVAL, "bad arguments");
  *bytes = size_t(s->nmom) * s->plane_bytes_state();
  return STARMAP_OK;
}

int starmap_get_state(const starmap_solver* cs, void* host_buf, size_t bytes, double* t, int64_t* step) {
  starmap_solver* s = const_cast<starmap_solver*>(cs);
  if (!s || !host_buf) return fail(STARMAP_EINVAL, "bad arguments");
  size_t need = size_t(s->nmom) * s->plane_bytes_state();
  if (bytes < need) return fail(STARMAP_EINVAL, "checkpoint buffer too small");
  int rc = ensure_device(s);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(host_buf, dptr(s, s->off_state), need, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (t) *t = s->t;
  if (step) *step = s->steps_done;
  return STARMAP_OK;
}

int starmap_set_state(starmap_solver* s, const void* host_buf, size_t bytes, double t, int64_t step) {
  if (!s || !host_buf) return fail(STARMAP_EINVAL, "bad arguments");
  size_t need = size_t(s->nmom) * s->plane_bytes_state();
  if (bytes != need) return fail(STARMAP_EINVAL, "checkpoint size does not match this solver");
  if (step < 0 || step > s->steps_total) return fail(STARMAP_EINVAL, "step out of range");
  int rc = ensure_device(s);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(dptr(s, s->off_state), host_buf, need, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->t = t;
  s->steps_done = step;
  if (s->time_dependent) s->materials_ready = false;
  return STARMAP_OK;
}

int starmap_diagnostics(const starmap_solver* cs, double* mass, double* l2, double* maxabs, int32_t* nonfinite) {
  starmap_solver* s = const_cast<starmap_solver*>(cs);
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  int rc = ensure_device(s);
  if (rc) return rc;
  DiagArgs a;
  a.u = dptr(s, s->off_state);
  size_t geo = s->off_diag + align256(size_t(s->diag_nblocks) * 4 * 8) + 256;
  a.plane_nx = reinterpret_cast<const int*>(dptr(s, geo));
  a.plane_ny = reinterpret_cast<const int*>(dptr(s, geo)) + s->nmom;
  a.nplanes = s->nmom;
  a.plane_stride = s->plane_stride;
  a.pitch = s->pitch;
  a.rows_per_block = s->diag_rows_per_block;
  a.blocks_per_plane = (s->ny + 1 + s->diag_rows_per_block - 1) / s->diag_rows_per_block;
  a.part = reinterpret_cast<double*>(dptr(s, s->off_diag));
  a.out = reinterpret_cast<double*>(dptr(s, s->off_diag + align256(size_t(s->diag_nblocks) * 4 * 8)));
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

int starmap_variant_count(void) { return sweep_variant_count(); }

int starmap_set_variant(starmap_solver* s, int32_t v) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (v < -1 || v >= sweep_variant_count()) return fail(STARMAP_EINVAL, "unknown variant");
  if (v >= 0) {
    int dev = 0, max_lds = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess) {
      int x = 0;
      if (hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && x > 0) max_lds = x;
    }
    if (sweep_lds_bytes(v, s->slots, s->storage) > size_t(max_lds))
      return fail(STARMAP_EINVAL, "tile variant does not fit the LDS for this moment order");
  }
  s->variant = v;
  if (s->device_ready) {
    if (v < 0) {
      v = default_variant(s);
      s->variant = v;
    }
    return upload_program(s);
  }
  return STARMAP_OK;
}

int starmap_set_graphs(starmap_solver* s, int32_t enable) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  s->use_graphs = enable != 0;
  if (!s->use_graphs) drop_pair_graphs(s);
  return STARMAP_OK;
}

int starmap_set_range_width(starmap_solver* s, int32_t width) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (std::find(std::begin(kChunkWidths), std::end(kChunkWidths), width) == std::end(kChunkWidths))
    return fail(STARMAP_EINVAL, "unsupported m-range width");
  const int keep = s->chunk_width;
  s->chunk_width = width;
  s->nchunks = sweep_chunk_count(s->N, width);
  if (!s->device_ready) return STARMAP_OK;
  int rc = upload_program(s);
  if (!rc && sweep_lds_bytes(s->variant, s->slots, s->storage) > size_t(max_lds_bytes()))
    rc = fail(STARMAP_EINVAL, "the tile variant does not fit the LDS at this m-range width");
  if (rc) {
    s->chunk_width = keep;
    (void)upload_program(s);
  }
  return rc;
}

int starmap_get_range_width(const starmap_solver* s, int32_t* width) {
  if (!s || !width) return fail(STARMAP_EINVAL, "bad arguments");
  *width = s->chunk_width;
  return STARMAP_OK;
}

int starmap_get_variant(const starmap_solver* s, int32_t* v, int32_t* tx, int32_t* ty) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (v) *v = s->variant;
  if (s->variant >= 0) {
    TileShape t = sweep_variant(s->variant);
    if (tx) *tx = t.tx;
    if (ty) *ty = t.ty;
  } else {
    if (tx) *tx = 0;
    if (ty) *ty = 0;
  }
  return STARMAP_OK;
}

int starmap_autotune(starmap_solver* s, int32_t sweeps) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (sweeps < 1) sweeps = 1;
  int rc = ensure_device(s);
  if (rc) return rc;
  if (!s->materials_ready) {
    rc = ensure_materials(s, s->t + 0.5 * s->dt);
    if (rc) return rc;
  }
  int dev = 0, max_lds = 64 * 1024;
  HIP_TRY(hipGetDevice(&dev));
  {
    int x = 0;
    if (hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && x > 0) max_lds = x;
  }
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int best = -1, best_w = s->chunk_width;
  float best_ms = 0.f;
  const int keep = s->variant, keep_w = s->chunk_width;
  std::vector<int> tried;
  for (int w : kChunkWidths) {
    if (rc) break;
    const int nch = sweep_chunk_count(s->N, w);
    if (std::find(tried.begin(), tried.end(), nch) != tried.end()) continue;  // same split as a narrower width
    tried.push_back(nch);
    s->chunk_width = w;
    for (int v = 0; v < sweep_variant_count() && !rc; ++v) {
      s->variant = v;
      // slots depend on the width: build first, then check the LDS
      rc = upload_program(s);
      if (rc) break;
      if (sweep_lds_bytes(v, s->slots, s->storage) > size_t(max_lds)) continue;
      // tau = 0 leaves every value unchanged (u + 0 * r = u), so timing on the
      // live state is harmless
      rc = sweep(s, 0, 0.0, false);
      if (!rc) rc = sweep(s, 1, 0.0, false);
      if (rc) break;
      HIP_TRY(hipEventRecord(e0, s->stream));
      for (int i = 0; i < sweeps && !rc; ++i) {
        rc = sweep(s, 0, 0.0, false);
        if (!rc) rc = sweep(s, 1, 0.0, false);
      }
      if (rc) break;
      HIP_TRY(hipEventRecord(e1, s->stream));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      if (std::getenv("STARMAP_VERBOSE")) {
        const TileShape ts = sweep_variant(v);
        std::fprintf(stderr, "starmap autotune: width %d variant %d (%dx%d) %.3f ms per sweep pair\n", w, v, ts.tx,
                     ts.ty, ms / sweeps);
      }
      if (best < 0 || ms < best_ms) {
        best = v;
        best_w = w;
        best_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    s->variant = keep;
    s->chunk_width = keep_w;
    (void)upload_program(s);
    return rc;
  }
  if (best < 0) return fail(STARMAP_ENOMEM, "no sweep tile fits the LDS for this moment order");
  s->variant = best;
  s->chunk_width = best_w;
  rc = upload_program(s);
  if (rc) return rc;
  if (const char* path = std::getenv("STARMAP_TUNE_CACHE")) {
    std::ofstream f(path, std::ios::app);
    f << s->N << " " << s->nx << " " << s->ny << " " << s->storage << " " << best << " " << best_w << "\n";
  }
  return STARMAP_OK;
}

int starmap_sweep_bytes(const starmap_solver* s, int32_t parity, double* bytes) {
  if (!s || !bytes || (parity != 0 && parity != 1)) return fail(STARMAP_EINVAL, "bad arguments");
  *bytes = sweep_bytes_of(s, parity);
  return STARMAP_OK;
}

int starmap_profile_begin(starmap_solver* s) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  s->profiling = true;
  s->ev_used = 0;
  s->prof_bytes = 0.0;
  return STARMAP_OK;
}

int starmap_profile_end(starmap_solver* s, double* kernel_ms, int64_t* launches, double* bytes) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  double ms = 0.0;
  if (s->ev_used) {
    HIP_TRY(hipEventSynchronize(s->ev[s->ev_used - 1]));
    for (size_t i = 0; i + 1 < s->ev_used; i += 2) {
      float m = 0.f;
      HIP_TRY(hipEventElapsedTime(&m, s->ev[i], s->ev[i + 1]));
      ms += m;
    }
  }
  if (kernel_ms) *kernel_ms = ms;
  if (launches) *launches = int64_t(s->ev_used / 2);
  if (bytes) *bytes = s->prof_bytes;
  s->profiling = false;
  s->ev_used = 0;
  s->prof_bytes = 0.0;
  return STARMAP_OK;
}

}  // extern "C"

namespace starmap {
namespace detail {

double sweep_bytes_of(const starmap_solver* s, int parity) {
  double b = 0.0;
  for (int k = 0; k < s->nmom; ++k) {
    const double pts = double(points_x(s, s->moms[k].gx)) * points_y(s, s->moms[k].gy);
    const bool even = s->moms[k].gx == s->moms[k].gy;
    const bool out = (parity == 0) == even;
    b += pts * double(s->ssize) * (out ? 2.0 : 1.0);
  }
  // decay planes of the outputs' grids (one read per point and plane used)
  std::vector<bool> used(size_t(s->dmap.nplanes), false);
  std::vector<bool> src_used(size_t(std::max(s->nsrc, 1)), false);
  for (int k = 0; k < s->nmom; ++k) {
    const bool even = s->moms[k].gx == s->moms[k].gy;
    if ((parity == 0) != even) continue;
    used[s->dmap.dk[k]] = true;
    if (s->qk[k] >= 0) src_used[s->qk[k]] = true;
  }
  for (int p = 0; p < s->dmap.nplanes; ++p)
    if (used[p]) b += double(points_x(s, s->dmap.plane_gx[p])) * points_y(s, s->dmap.plane_gy[p]) * s->csize;
  for (int k = 0; k < s->nmom; ++k)
    if (s->qk[k] >= 0 && src_used[s->qk[k]])
      b += double(points_x(s, s->moms[k].gx)) * points_y(s, s->moms[k].gy) * s->ssize;
  return b;
}

}  // namespace detail
}  // namespace starmap

extern "C" const char* starmap_last_error(void) { return g_last_error.c_str(); }

extern "C" int starmap_reset(starmap_solver* s) {
  if (!s) return fail(STARMAP_EINVAL, "solver is NULL");
  if (s->device_ready) {
    int rc = upload_initial(s);
    if (rc) return rc;
  }
  s->t = 0.0;
  s->steps_done = 0;
  if (s->time_dependent) s->materials_ready = false;
  return STARMAP_OK;
}

// ------------------------------------------------------------ batches
// A batch advances several independent solvers together: every sweep number
// j of the fused composition is one launch per group of instances over the
// workgroups of the group's instances still running, and the whole run is one
// HIP graph.  Instances are grouped by moment order N; each group has its own
// tile variant and m-range width (the autotuner picks them per group).

namespace starmap {
namespace detail {
struct BatchGroup {
  int N = 0;
  std::vector<int> members;  // instance indices, in the caller's order
  int variant = -1, width = 0, slots = 0;
  bool tiles_set = false;
};
// One launch per sweep over the running instances of a plan: a group, or with
// merged launches every instance (one tile variant for all groups).
struct BatchPlan {
  int variant = 0, slots = 0;
  std::vector<int> members;  // instances the plan covers
  std::vector<int> order;    // members with sweeps left, by sweeps (descending, stable)
  std::vector<int> nsweeps;
  std::vector<int> first;    // workgroup prefix (order.size() + 1 values)
  size_t tab0 = 0;           // first table entry of the plan
  size_t first0 = 0;         // first prefix value of the plan in the table's int array
};
}  // namespace detail
}  // namespace starmap

struct starmap_batch {
  std::vector<starmap_solver*> inst;  // as given by the caller
  int storage = STORE_FP64;
  std::vector<starmap::detail::BatchGroup> groups;  // by ascending N
  // merged: one launch per sweep over the instances of every group (all
  // groups on one tile variant); else one launch per sweep and group, each
  // group's launches a chain on its own stream
  bool merged = false;
  std::vector<starmap::detail::BatchPlan> plans;  // of the current table
  hipStream_t stream = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  // one stream per group: a run forks from `stream` into the groups' chains
  // of launches (independent instances) and joins back
  std::vector<hipStream_t> gstream;
  std::vector<hipEvent_t> gdone;
  hipEvent_t fork = nullptr;
  void* dtab = nullptr;  // BatchEntry[count], then the groups' workgroup prefixes
  // batches of closure solvers (one group, N = 5): ClosureInst[count], then
  // int cfirst[count + 1] (evaluation blocks of the closure sweep per
  // instance, in the group's order)
  bool closure = false;
  // closure batches: the solvers' setting (starmap_closure_set_fused), read at
  // every run: one fused kernel per odd sweep, or the network then a batched
  // odd sweep
  bool closure_fused = false;
  void* ctab = nullptr;
  std::vector<int> cfirst;
  // captured run
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> graph_key;
  // last run
  double last_ms = 0.0, last_bytes = 0.0;
  int64_t last_updates = 0, last_launches = 0;
};

namespace starmap {
namespace detail {

size_t batch_table_bytes(int count, int ngroups) {
  return align256(size_t(count) * sizeof(BatchEntry)) + size_t(count + ngroups) * 4;
}
size_t closure_table_bytes(int count) {
  return align256(size_t(count) * sizeof(ClosureInst)) + size_t(count + 1) * 4;
}
int closure_blocks_of(const starmap_solver* s) { return ((s->nx + 1) * (s->ny + 1) + 63) / 64; }

int max_lds_bytes() {
  int dev = 0, max_lds = 64 * 1024;
  if (hipGetDevice(&dev) == hipSuccess) {
    int x = 0;
    if (hipDeviceGetAttribute(&x, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && x > 0) max_lds = x;
  }
  return max_lds;
}

void drop_graph(starmap_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_key.clear();
}

// Device workspaces and materials of every instance.
int batch_devices(starmap_batch* b) {
  for (auto* s : b->inst) {
    int rc = ensure_device(s);
    if (rc) return rc;
    if (!s->materials_ready) {
      rc = upload_materials(s, s->t + 0.5 * s->dt);
      if (rc) return rc;
    }
  }
  return STARMAP_OK;
}

// The tile of one group: every member's programs for it, the group's LDS.
int group_prepare(starmap_batch* b, BatchGroup& g, int variant, int width) {
  int rc = batch_devices(b);
  if (rc) return rc;
  if (g.tiles_set && variant == g.variant && width == g.width) return STARMAP_OK;
  int slots = 0;
  for (int i : g.members) {
    starmap_solver* s = b->inst[i];
    s->variant = variant;
    s->chunk_width = width;
    rc = upload_program(s);
    if (rc) return rc;
    if (s->prog[0].chunks.size() != s->prog[1].chunks.size())
      return fail(STARMAP_ESTATE, "sweep programs of the two parities differ in m ranges");
    slots = std::max(slots, s->slots);
  }
  g.tiles_set = true;
  g.variant = variant;
  g.width = width;
  g.slots = slots;
  drop_graph(b);
  if (sweep_lds_bytes(variant, slots, b->storage) > size_t(max_lds_bytes()))
    return fail(STARMAP_EINVAL, "tile variant does not fit the LDS for the moment order of a batch group");
  HIP_TRY(prepare_sweep(b->storage, variant, slots));
  return STARMAP_OK;
}

// ... every group with the same tile, or the default tile where none is set.
int batch_prepare(starmap_batch* b, int variant, int width) {
  for (auto& g : b->groups) {
    int rc = group_prepare(b, g, variant, width);
    if (rc) return rc;
  }
  return STARMAP_OK;
}

int batch_ready(starmap_batch* b) {
  for (auto& g : b->groups) {
    int rc = group_prepare(b, g, g.tiles_set ? g.variant : 0, g.tiles_set ? g.width : kDefaultChunkWidth);
    if (rc) return rc;
  }
  return STARMAP_OK;
}

int items_of(const starmap_solver* s) {
  const TileShape ts = sweep_variant(s->variant);
  const int ntx = (s->nx + 1 + ts.tx - 1) / ts.tx, nty = (s->ny + 1 + ts.ty - 1) / ts.ty;
  return ntx * nty * int(s->prog[0].chunks.size());
}

// Per launch plan, the entries of the members with sweeps[i] > 0 sorted by
// sweeps (descending, stable), uploaded with the plan's workgroup prefix.
// zero_tau: every sub-step length 0 (timing on live state leaves it unchanged).
int batch_table(starmap_batch* b, const std::vector<int>& sweeps, bool zero_tau) {
  const int count = int(b->inst.size());
  const int ng = int(b->groups.size());
  if (b->closure) {
    b->closure_fused = b->inst[0]->closure_fused;
    for (const auto* s : b->inst)
      if (s->closure_fused != b->closure_fused)
        return fail(STARMAP_EINVAL, "the closure solvers of a batch must agree on starmap_closure_set_fused");
  }
  b->plans.clear();
  if (b->merged && ng > 1) {
    BatchPlan pl;
    pl.variant = b->groups[0].variant;
    for (const auto& g : b->groups) {
      if (g.variant != pl.variant) return fail(STARMAP_ESTATE, "merged batch launches need one tile variant");
      pl.slots = std::max(pl.slots, g.slots);
      pl.members.insert(pl.members.end(), g.members.begin(), g.members.end());
    }
    b->plans.push_back(pl);
  } else {
    for (const auto& g : b->groups) {
      BatchPlan pl;
      pl.variant = g.variant;
      pl.slots = g.slots;
      pl.members = g.members;
      b->plans.push_back(pl);
    }
  }
  if (b->merged && ng > 1) HIP_TRY(prepare_sweep(b->storage, b->plans[0].variant, b->plans[0].slots));
  std::vector<BatchEntry> tab;
  std::vector<int> firsts;
  for (auto& g : b->plans) {
    std::vector<int> ord;
    for (int i : g.members)
      if (sweeps[i] > 0) ord.push_back(i);
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sweeps[x] > sweeps[y]; });
    g.tab0 = tab.size();
    g.first0 = firsts.size();
    g.order = ord;
    g.nsweeps.assign(ord.size(), 0);
    g.first.assign(ord.size() + 1, 0);
    int64_t total = 0;
    for (size_t r = 0; r < ord.size(); ++r) {
      starmap_solver* s = b->inst[ord[r]];
      BatchEntry e;
      std::memset(&e, 0, sizeof(e));
      e.u = dptr(s, s->off_state);
      e.decay = dptr(s, s->off_decay);
      for (int p = 0; p < 2; ++p) {
        const auto& pr = s->prog[p];
        char* base = dptr(s, s->off_prog[p]);
        size_t o = 0;
        e.chunks[p] = reinterpret_cast<const int4*>(base + o);
        o += align256(pr.chunks.size() * 16);
        e.orders[p] = reinterpret_cast<const int4*>(base + o);
        o += align256(pr.orders.size() * 16);
        e.loads[p] = reinterpret_cast<const int4*>(base + o);
        o += align256(pr.loads.size() * 16);
        e.rows[p] = reinterpret_cast<const int*>(base + o);
        o += align256(pr.rows.size() * 64);
        e.rcoef[p] = base + o;
        e.zero_off[p] = pr.zero_off;
      }
      e.plane_stride = s->plane_stride;
      e.tau_full = zero_tau ? 0.0 : s->dt;
      e.tau_half = zero_tau ? 0.0 : 0.5 * s->dt;
      e.pitch = s->pitch;
      e.nx = s->nx;
      e.ny = s->ny;
      e.px = s->px;
      e.py = s->py;
      const TileShape ts = sweep_variant(s->variant);
      e.ntx = (s->nx + 1 + ts.tx - 1) / ts.tx;
      e.nty = (s->ny + 1 + ts.ty - 1) / ts.ty;
      e.nchunks = int(s->prog[0].chunks.size());
      e.nsweeps = sweeps[ord[r]];
      e.strip = s->tile_strip;
      e.even_b_delta = (s->closure && b->closure_fused) ? int64_t(s->off_prog_b) - int64_t(s->off_prog[0]) : 0;
      tab.push_back(e);
      g.nsweeps[r] = sweeps[ord[r]];
      g.first[r] = int(total);
      total += items_of(s);
    }
    if (total >= (int64_t(1) << 31)) return fail(STARMAP_EINVAL, "too many workgroups in one batched sweep");
    g.first[ord.size()] = int(total);
    firsts.insert(firsts.end(), g.first.begin(), g.first.end());
  }
  std::vector<char> buf(batch_table_bytes(count, ng), 0);
  std::memcpy(buf.data(), tab.data(), tab.size() * sizeof(BatchEntry));
  std::memcpy(buf.data() + align256(size_t(count) * sizeof(BatchEntry)), firsts.data(), firsts.size() * 4);
  HIP_TRY(hipMemcpyAsync(b->dtab, buf.data(), buf.size(), hipMemcpyHostToDevice, b->stream));
  if (b->closure) {
    // the closure sweep's instances in the (single) group's order, with their block prefix
    const BatchPlan& g = b->plans[0];
    std::vector<ClosureInst> ct(g.order.size());
    std::vector<int> cf(g.order.size() + 1, 0);
    int64_t nb = 0;
    for (size_t r = 0; r < g.order.size(); ++r) {
      starmap_solver* s = b->inst[g.order[r]];
      ClosureInst& c = ct[r];
      std::memset(&c, 0, sizeof(c));
      const size_t pb = s->plane_bytes_state();
      c.u = dptr(s, s->off_state);
      c.a5 = dptr(s, s->off_state + size_t(closure_plane_a(s)) * pb);
      c.b5 = dptr(s, s->off_state + size_t(closure_plane_b(s)) * pb);
      c.decay = dptr(s, s->off_decay);
      c.tau_full = zero_tau ? 0.0 : s->dt;
      c.tau_half = zero_tau ? 0.0 : 0.5 * s->dt;
      c.nsweeps = sweeps[g.order[r]];
      c.G = s->cgeo;
      c.odd = s->codd;
      cf[r] = int(nb);
      nb += closure_blocks_of(s);
    }
    if (nb >= (int64_t(1) << 31)) return fail(STARMAP_EINVAL, "too many closure blocks in one batched sweep");
    cf[g.order.size()] = int(nb);
    std::vector<char> cb(closure_table_bytes(count), 0);
    std::memcpy(cb.data(), ct.data(), ct.size() * sizeof(ClosureInst));
    std::memcpy(cb.data() + align256(size_t(count) * sizeof(ClosureInst)), cf.data(), cf.size() * 4);
    HIP_TRY(hipMemcpyAsync(b->ctab, cb.data(), cb.size(), hipMemcpyHostToDevice, b->stream));
    b->cfirst = cf;
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  return STARMAP_OK;
}

// Queue sweeps j0 .. j1-1 of the current table on the batch stream: one
// launch per plan with instances still running (only plan `only` if >= 0).
int batch_launch(starmap_batch* b, int j0, int j1, int only = -1) {
  const BatchEntry* tab = reinterpret_cast<const BatchEntry*>(b->dtab);
  const int* firsts =
      reinterpret_cast<const int*>(static_cast<char*>(b->dtab) + align256(b->inst.size() * sizeof(BatchEntry)));
  for (int j = j0; j < j1; ++j) {
    if (b->closure && (j & 1) == 0) {
      // odd sweep of closure solvers: the network and the odd update in one
      // kernel, or the network alone here and the odd sweep below
      const BatchPlan& g = b->plans[0];
      int na = int(g.nsweeps.size());
      while (na > 0 && g.nsweeps[na - 1] <= j) --na;
      if (na == 0) continue;
      const ClosureInst* ct = reinterpret_cast<const ClosureInst*>(b->ctab);
      const int* cf = reinterpret_cast<const int*>(static_cast<char*>(b->ctab) +
                                                   align256(b->inst.size() * sizeof(ClosureInst)));
      const starmap_solver* s0 = b->inst[g.order[0]];
      const ClosureNet* net = reinterpret_cast<const ClosureNet*>(dptr(s0, s0->off_net));
      if (b->closure_fused) {
        HIP_TRY(launch_closure_batch(b->storage, ct, cf, na, b->cfirst[na], j, net, b->stream));
        continue;
      }
      HIP_TRY(launch_closure_batch_net(b->storage, ct, cf, na, b->cfirst[na], net, b->stream));
    }
    for (int gi = 0; gi < int(b->plans.size()); ++gi) {
      if (only >= 0 && gi != only) continue;
      const BatchPlan& g = b->plans[gi];
      int na = int(g.nsweeps.size());
      while (na > 0 && g.nsweeps[na - 1] <= j) --na;
      if (na == 0) continue;
      HIP_TRY(launch_sweep_batch(b->storage, g.variant, tab + g.tab0, firsts + g.first0, na, g.first[na], j,
                                 g.slots, b->stream));
    }
  }
  return STARMAP_OK;
}

// Cell-moment work of a group for one step of every member (for reporting the
// dominant group's tile).
double group_work(const starmap_batch* b, const BatchGroup& g) {
  double w = 0.0;
  for (int i : g.members) {
    const starmap_solver* s = b->inst[i];
    w += double(s->nmom) * s->nx * s->ny * double(s->steps_total);
  }
  return w;
}

// Cell-moment work of a plan's members for a whole run.
double plan_work(const starmap_batch* b, const BatchPlan& g) {
  double w = 0.0;
  for (int i : g.members) {
    const starmap_solver* s = b->inst[i];
    w += double(s->nmom) * s->nx * s->ny * double(s->steps_total);
  }
  return w;
}

// Sweeps j0 .. j1-1 of the current table: a single plan (or a closure batch)
// on the batch stream; several plans each as a chain on its own stream, forked
// from and joined back into the batch stream, so that one group's launches
// fill the machine while another's drain.
int batch_launch_all(starmap_batch* b, int j0, int j1) {
  if (b->closure || b->plans.size() == 1) return batch_launch(b, j0, j1);
  const BatchEntry* tab = reinterpret_cast<const BatchEntry*>(b->dtab);
  const int* firsts =
      reinterpret_cast<const int*>(static_cast<char*>(b->dtab) + align256(b->inst.size() * sizeof(BatchEntry)));
  // the plans with the most work first: the chains start one after another
  // as the machine frees up, and the longest one bounds the run
  std::vector<int> ord(b->plans.size());
  for (size_t gi = 0; gi < ord.size(); ++gi) ord[gi] = int(gi);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int x, int y) { return plan_work(b, b->plans[x]) > plan_work(b, b->plans[y]); });
  HIP_TRY(hipEventRecord(b->fork, b->stream));
  for (int gi : ord) HIP_TRY(hipStreamWaitEvent(b->gstream[gi], b->fork, 0));
  // submitted sweep by sweep across the plans (a chain submitted whole could
  // fill its queue and hold back the next)
  for (int j = j0; j < j1; ++j)
    for (int gi : ord) {
      const BatchPlan& g = b->plans[gi];
      int na = int(g.nsweeps.size());
      while (na > 0 && g.nsweeps[na - 1] <= j) --na;
      if (na == 0) continue;
      HIP_TRY(launch_sweep_batch(b->storage, g.variant, tab + g.tab0, firsts + g.first0, na, g.first[na], j,
                                 g.slots, b->gstream[gi]));
    }
  for (size_t gi = 0; gi < b->plans.size(); ++gi) {
    HIP_TRY(hipEventRecord(b->gdone[gi], b->gstream[gi]));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->gdone[gi], 0));
  }
  return STARMAP_OK;
}

int batch_sync_solvers(starmap_batch* b) {
  for (auto* s : b->inst) HIP_TRY(hipStreamSynchronize(s->stream));
  return STARMAP_OK;
}

}  // namespace detail
}  // namespace starmap

extern "C" {

int starmap_batch_create(starmap_solver* const* solvers, int32_t count, starmap_batch** out) {
  if (!out) return fail(STARMAP_EINVAL, "out is NULL");
  *out = nullptr;
  if (!solvers || count < 1) return fail(STARMAP_EINVAL, "empty batch");
  std::vector<starmap_solver*> v(solvers, solvers + count);
  for (int i = 0; i < count; ++i) {
    if (!v[i]) return fail(STARMAP_EINVAL, "NULL solver in batch");
    if (v[i]->time_dependent || v[i]->separable)
      return fail(STARMAP_EINVAL, "batched solvers need time-independent data");
    if (v[i]->has_diffusion) return fail(STARMAP_EINVAL, "batched solvers cannot take the D_N diffusion step");
    if (v[i]->closure != v[0]->closure)
      return fail(STARMAP_EINVAL, "a batch holds closure solvers only or none");
    if (v[i]->closure && !v[i]->closure_loaded)
      return fail(STARMAP_EINVAL, "batched closure solvers need a loaded network");
    if (v[i]->closure && v[i]->closure_w != v[0]->closure_w)
      return fail(STARMAP_EINVAL, "batched closure solvers need one network");
    if (v[i]->storage != v[0]->storage) return fail(STARMAP_EINVAL, "batched solvers need one storage precision");
  }
  {
    std::vector<starmap_solver*> u = v;
    std::sort(u.begin(), u.end());
    if (std::adjacent_find(u.begin(), u.end()) != u.end()) return fail(STARMAP_EINVAL, "solver listed twice");
  }
  auto b = std::make_unique<starmap_batch>();
  b->inst = v;
  b->storage = v[0]->storage;
  b->closure = v[0]->closure;
  {
    std::vector<int> orders;
    for (auto* s : v) orders.push_back(s->N);
    std::sort(orders.begin(), orders.end());
    orders.erase(std::unique(orders.begin(), orders.end()), orders.end());
    for (int N : orders) {
      BatchGroup g;
      g.N = N;
      for (int i = 0; i < count; ++i)
        if (v[i]->N == N) g.members.push_back(i);
      b->groups.push_back(g);
    }
  }
  HIP_TRY(hipStreamCreate(&b->stream));
  HIP_TRY(hipEventCreate(&b->ev[0]));
  HIP_TRY(hipEventCreate(&b->ev[1]));
  if (!b->closure && b->groups.size() > 1) {
    HIP_TRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    b->gstream.assign(b->groups.size(), nullptr);
    b->gdone.assign(b->groups.size(), nullptr);
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
      HIP_TRY(hipStreamCreate(&b->gstream[gi]));
      HIP_TRY(hipEventCreateWithFlags(&b->gdone[gi], hipEventDisableTiming));
    }
  }
  HIP_TRY(hipMalloc(&b->dtab, batch_table_bytes(count, int(b->groups.size()))));
  if (b->closure) HIP_TRY(hipMalloc(&b->ctab, closure_table_bytes(count)));
  *out = b.release();
  return STARMAP_OK;
}

void starmap_batch_destroy(starmap_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (auto st : b->gstream)
    if (st) (void)hipStreamSynchronize(st);
  drop_graph(b);
  if (b->dtab) (void)hipFree(b->dtab);
  if (b->ctab) (void)hipFree(b->ctab);
  for (auto& e : b->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto e : b->gdone)
    if (e) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (auto st : b->gstream)
    if (st) (void)hipStreamDestroy(st);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

int starmap_batch_set_variant(starmap_batch* b, int32_t variant, int32_t width) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  if (variant < 0 || variant >= sweep_variant_count()) return fail(STARMAP_EINVAL, "unknown variant");
  if (std::find(std::begin(kChunkWidths), std::end(kChunkWidths), width) == std::end(kChunkWidths))
    return fail(STARMAP_EINVAL, "unsupported m-range width");
  return batch_prepare(b, variant, width);
}

int starmap_batch_set_group_variant(starmap_batch* b, int32_t group, int32_t variant, int32_t width) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  if (group < 0 || group >= int32_t(b->groups.size())) return fail(STARMAP_EINVAL, "group out of range");
  if (variant < 0 || variant >= sweep_variant_count()) return fail(STARMAP_EINVAL, "unknown variant");
  if (std::find(std::begin(kChunkWidths), std::end(kChunkWidths), width) == std::end(kChunkWidths))
    return fail(STARMAP_EINVAL, "unsupported m-range width");
  int rc = batch_ready(b);
  if (rc) return rc;
  // merged launches stay on while every group keeps one variant
  if (b->merged && b->groups.size() > 1 && variant != b->groups[group == 0 ? 1 : 0].variant) b->merged = false;
  return group_prepare(b, b->groups[group], variant, width);
}

int starmap_batch_get_variant(const starmap_batch* b, int32_t* variant, int32_t* width) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  // the group with the most cell-moment work
  const BatchGroup* best = nullptr;
  double wmax = -1.0;
  for (const auto& g : b->groups) {
    const double w = group_work(b, g);
    if (w > wmax) {
      wmax = w;
      best = &g;
    }
  }
  if (variant) *variant = best && best->tiles_set ? best->variant : -1;
  if (width) *width = best && best->tiles_set ? best->width : 0;
  return STARMAP_OK;
}

int starmap_batch_group_count(const starmap_batch* b) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  return int(b->groups.size());
}

int starmap_batch_get_group(const starmap_batch* b, int32_t group, int32_t* N, int32_t* count, int32_t* variant,
                            int32_t* width) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  if (group < 0 || group >= int32_t(b->groups.size())) return fail(STARMAP_EINVAL, "group out of range");
  const BatchGroup& g = b->groups[group];
  if (N) *N = g.N;
  if (count) *count = int32_t(g.members.size());
  if (variant) *variant = g.tiles_set ? g.variant : -1;
  if (width) *width = g.tiles_set ? g.width : 0;
  return STARMAP_OK;
}

int starmap_batch_run(starmap_batch* b, int32_t use_graph) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  int rc = batch_ready(b);
  if (rc) return rc;
  rc = batch_sync_solvers(b);
  if (rc) return rc;
  const int count = int(b->inst.size());
  std::vector<int> sweeps(count);
  int64_t updates = 0;
  double bytes = 0.0;
  for (int i = 0; i < count; ++i) {
    starmap_solver* s = b->inst[i];
    const int64_t n = s->steps_total - s->steps_done;
    if (2 * n + 1 >= (int64_t(1) << 31)) return fail(STARMAP_EINVAL, "too many steps for one batched run");
    sweeps[i] = n > 0 ? int(2 * n + 1) : 0;
    updates += int64_t(s->nmom) * s->nx * s->ny * n;
    if (n > 0) bytes += double(n + 1) * sweep_bytes_of(s, 1) + double(n) * sweep_bytes_of(s, 0);
  }
  rc = batch_table(b, sweeps, false);
  if (rc) return rc;
  int jmax = 0;
  int64_t launches = 0;
  for (const auto& g : b->plans) {
    if (!g.nsweeps.empty()) jmax = std::max(jmax, g.nsweeps[0]);
    for (int j = 0; !g.nsweeps.empty() && j < g.nsweeps[0]; ++j)
      if (!(b->closure && b->closure_fused && (j & 1) == 0)) ++launches;
  }
  // closure batches: one network launch (fused: network and odd sweep) per odd sweep
  if (b->closure && !b->plans[0].nsweeps.empty()) launches += (b->plans[0].nsweeps[0] + 1) / 2;
  HIP_TRY(hipEventRecord(b->ev[0], b->stream));
  if (jmax > 0) {
    if (use_graph) {
      // the graph depends on every group's tile (kernel, LDS, programs) and
      // on the launch plans
      std::vector<int> key{b->merged ? 1 : 0, b->closure_fused ? 1 : 0};
      for (const auto& g : b->groups) key.insert(key.end(), {g.variant, g.width, g.slots});
      for (const auto& g : b->plans) {
        key.insert(key.end(), {g.variant, g.slots, int(g.nsweeps.size())});
        key.insert(key.end(), g.order.begin(), g.order.end());
        key.insert(key.end(), g.nsweeps.begin(), g.nsweeps.end());
        key.insert(key.end(), g.first.begin(), g.first.end());
      }
      if (!b->exec || key != b->graph_key) {
        drop_graph(b);
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        rc = batch_launch_all(b, 0, jmax);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->stream, &g);
        if (rc) {
          if (g) (void)hipGraphDestroy(g);
          return rc;
        }
        HIP_TRY(e);
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_key = key;
        // time the graph launch, not the capture
        HIP_TRY(hipEventRecord(b->ev[0], b->stream));
      }
      HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    } else {
      rc = batch_launch_all(b, 0, jmax);
      if (rc) return rc;
    }
  }
  HIP_TRY(hipEventRecord(b->ev[1], b->stream));
  HIP_TRY(hipEventSynchronize(b->ev[1]));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
  if (b->closure) {
    const BatchPlan& g = b->plans[0];
    for (size_t r = 0; r < g.order.size(); ++r) {
      starmap_solver* s = b->inst[g.order[r]];
      // fused: (nsweeps + 1) / 2 odd sweeps each moved the order-5 moments once
      s->c5_flip = b->closure_fused ? ((g.nsweeps[r] + 1) / 2) & 1 : 0;
      rc = closure_settle(s);
      if (rc) return rc;
      HIP_TRY(hipStreamSynchronize(s->stream));
    }
  }
  for (auto* s : b->inst) {
    s->steps_done = s->steps_total;
    s->t = double(s->steps_done) * s->dt;
  }
  b->last_ms = ms;
  b->last_updates = updates;
  b->last_bytes = bytes;
  b->last_launches = launches;
  return STARMAP_OK;
}

int starmap_batch_last_run(const starmap_batch* b, double* ms, int64_t* updates, double* bytes, int64_t* launches) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  if (ms) *ms = b->last_ms;
  if (updates) *updates = b->last_updates;
  if (bytes) *bytes = b->last_bytes;
  if (launches) *launches = b->last_launches;
  return STARMAP_OK;
}

int starmap_batch_autotune(starmap_batch* b, int32_t sweeps) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  if (sweeps < 1) sweeps = 1;
  const int count = int(b->inst.size());
  const int ng = int(b->groups.size());
  const int max_lds = max_lds_bytes();
  {
    int rc = batch_ready(b);
    if (rc) return rc;
  }
  const bool verbose = std::getenv("STARMAP_VERBOSE") != nullptr;
  b->merged = false;
  // each group on its own: every (width, variant) pair that fits, timed on a
  // sweep pair of the group's instances (tau = 0 leaves every value unchanged)
  std::vector<std::map<std::pair<int, int>, float>> times(ng);
  for (int gi = 0; gi < ng; ++gi) {
    BatchGroup& g = b->groups[gi];
    int best_v = -1, best_w = 0;
    float best_ms = 0.f;
    std::vector<int> tried;
    for (int w : kChunkWidths) {
      const int split = sweep_chunk_count(g.N, w);
      if (std::find(tried.begin(), tried.end(), split) != tried.end()) continue;  // same m ranges as a narrower width
      tried.push_back(split);
      for (int v = 0; v < sweep_variant_count(); ++v) {
        // LDS check before the kernels are opted in
        int slots = 0;
        for (int i : g.members) {
          starmap_solver* s = b->inst[i];
          s->variant = v;
          s->chunk_width = w;
          int rc = upload_program(s);
          if (rc) return rc;
          slots = std::max(slots, s->slots);
        }
        g.tiles_set = false;
        if (sweep_lds_bytes(v, slots, b->storage) > size_t(max_lds)) continue;
        int rc = group_prepare(b, g, v, w);
        if (rc) return rc;
        // three sweeps: odd, even, odd.  A closure batch times the first pair
        // (odd sweep 0 evaluates the network; fused, it also moves the order-5
        // moments into the closure planes, where even sweep 1 reads them)
        const int j0 = b->closure ? 0 : 1;
        rc = batch_table(b, std::vector<int>(count, 3), true);
        if (!rc) rc = batch_launch(b, j0, j0 + 2, gi);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->ev[0], b->stream));
        for (int i = 0; i < sweeps && !rc; ++i) rc = batch_launch(b, j0, j0 + 2, gi);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(b->ev[1], b->stream));
        HIP_TRY(hipEventSynchronize(b->ev[1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
        ms /= float(sweeps);
        times[gi][{v, w}] = ms;
        if (verbose) {
          const TileShape ts = sweep_variant(v);
          std::fprintf(stderr, "starmap batch autotune: N %d width %d variant %d (%dx%d) %.3f ms per sweep pair\n",
                       g.N, w, v, ts.tx, ts.ty, ms);
        }
        if (best_v < 0 || ms < best_ms) {
          best_v = v;
          best_w = w;
          best_ms = ms;
        }
      }
    }
    if (best_v < 0) return fail(STARMAP_ENOMEM, "no sweep tile fits the LDS for a group of this batch");
    int rc = group_prepare(b, g, best_v, best_w);
    if (rc) return rc;
  }
  if (b->closure || ng == 1) return STARMAP_OK;

  // the whole batch: the groups' best tiles as concurrent chains, against
  // merged launches on one variant (each group at its best width for it),
  // each timed on sweep pairs of every instance
  auto time_all = [&](float* out) -> int {
    int rc = batch_table(b, std::vector<int>(count, 3), true);
    if (!rc) rc = batch_launch_all(b, 1, 3);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b->ev[0], b->stream));
    for (int i = 0; i < sweeps && !rc; ++i) rc = batch_launch_all(b, 1, 3);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(b->ev[1], b->stream));
    HIP_TRY(hipEventSynchronize(b->ev[1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, b->ev[0], b->ev[1]));
    *out = ms / float(sweeps);
    return STARMAP_OK;
  };
  std::vector<std::pair<int, int>> chains(ng);
  for (int gi = 0; gi < ng; ++gi) chains[gi] = {b->groups[gi].variant, b->groups[gi].width};
  float best_ms = 0.f;
  int rc = time_all(&best_ms);
  if (rc) return rc;
  if (verbose) std::fprintf(stderr, "starmap batch autotune: groups as chains %.3f ms per sweep pair\n", best_ms);
  int best_merged_v = -1;
  // candidate variants: timed for every group, ranked by the sum of the
  // groups' best times on them
  std::vector<std::pair<float, int>> cand;
  for (int v = 0; v < sweep_variant_count(); ++v) {
    float sum = 0.f;
    bool all = true;
    for (int gi = 0; gi < ng && all; ++gi) {
      float bv = -1.f;
      for (const auto& kv : times[gi])
        if (kv.first.first == v && (bv < 0.f || kv.second < bv)) bv = kv.second;
      if (bv < 0.f) all = false; else sum += bv;
    }
    if (all) cand.push_back({sum, v});
  }
  std::sort(cand.begin(), cand.end());
  if (cand.size() > 2) cand.resize(2);
  std::vector<int> best_widths;
  for (const auto& c : cand) {
    const int v = c.second;
    std::vector<int> widths(ng);
    for (int gi = 0; gi < ng; ++gi) {
      float bv = -1.f;
      for (const auto& kv : times[gi])
        if (kv.first.first == v && (bv < 0.f || kv.second < bv)) {
          bv = kv.second;
          widths[gi] = kv.first.second;
        }
      rc = group_prepare(b, b->groups[gi], v, widths[gi]);
      if (rc) return rc;
    }
    b->merged = true;
    float ms = 0.f;
    rc = time_all(&ms);
    b->merged = false;
    if (rc) return rc;
    if (verbose) std::fprintf(stderr, "starmap batch autotune: merged on variant %d %.3f ms per sweep pair\n", v, ms);
    if (ms < best_ms) {
      best_ms = ms;
      best_merged_v = v;
      best_widths = widths;
    }
  }
  for (int gi = 0; gi < ng; ++gi) {
    rc = best_merged_v >= 0 ? group_prepare(b, b->groups[gi], best_merged_v, best_widths[gi])
                            : group_prepare(b, b->groups[gi], chains[gi].first, chains[gi].second);
    if (rc) return rc;
  }
  b->merged = best_merged_v >= 0;
  drop_graph(b);
  return STARMAP_OK;
}

int starmap_batch_set_merged(starmap_batch* b, int32_t merged) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  int rc = batch_ready(b);
  if (rc) return rc;
  if (merged)
    for (const auto& g : b->groups)
      if (g.variant != b->groups[0].variant)
        return fail(STARMAP_EINVAL, "merged batch launches need one tile variant for every group");
  b->merged = merged != 0;
  drop_graph(b);
  return STARMAP_OK;
}

int starmap_batch_get_merged(const starmap_batch* b) {
  if (!b) return fail(STARMAP_EINVAL, "batch is NULL");
  return b->merged ? 1 : 0;
}

}  // extern "C"
