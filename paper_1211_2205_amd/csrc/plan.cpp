// Host plan of the staggered-grid P_N step (Seibold & Frank, arXiv 1211.2205).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <stdexcept>
#include <tuple>

namespace starmap {

std::vector<MomentInfo> moment_list(int N) {
  // Sect. 3, eq. (transformation): u = (R_0^0, R_1^1, I_1^1, R_2^2, I_2^2, R_2^0, ...).
  // Lemma 2 fixes the grids: M_x couples R<->R and I<->I across adjacent orders,
  // M_y couples R<->I; with R_0^0 on G11 this places R of even order on G11,
  // R of odd order on G21, I of odd order on G12 and I of even order on G22.
  std::vector<MomentInfo> out;
  for (int l = 0; l <= N; ++l) {
    for (int m = l; m >= 0; m -= 2) {
      bool even = (l % 2) == 0;
      out.push_back({0, l, m, even ? 1 : 2, 1});
      if (m > 0) out.push_back({1, l, m, even ? 2 : 1, 2});
    }
  }
  return out;
}

int moment_count(int N) { return (N + 1) * (N + 2) / 2; }

namespace {

// Ladder coefficients of the spherical-harmonic recursion (Sect. 3).  With
// A(l,m) = c_l^m = f_{l+1}^{m+1} and B(l,m) = e_l^m = d_{l+1}^{m-1}, the
// complex x-row of psi_l^m couples
//   psi_{l+1}^{m+1} with -A(l,m)/2,      psi_{l-1}^{m+1} with  B(l-1,m+1)/2,
//   psi_{l+1}^{m-1} with  B(l,m)/2,      psi_{l-1}^{m-1} with -A(l-1,m-1)/2,
// and the y-row carries the same terms times +i (m+1 targets) and -i (m-1).
double ladder_A(int l, int m) {
  double num = double(l + m + 1) * double(l + m + 2);
  return num <= 0.0 ? 0.0 : std::sqrt(num / (double(2 * l + 1) * double(2 * l + 3)));
}
double ladder_B(int l, int m) {
  double num = double(l - m + 1) * double(l - m + 2);
  return num <= 0.0 ? 0.0 : std::sqrt(num / (double(2 * l + 1) * double(2 * l + 3)));
}
// alpha_plus(l, lp, m): coefficient of psi_{lp}^{m+1} in the x-row of psi_l^m.
double alpha_plus(int l, int lp, int m) {
  return lp == l + 1 ? -0.5 * ladder_A(l, m) : 0.5 * ladder_B(l - 1, m + 1);
}
// alpha_minus(l, lp, m): coefficient of psi_{lp}^{m-1} in the x-row of psi_l^m.
double alpha_minus(int l, int lp, int m) {
  return lp == l + 1 ? 0.5 * ladder_B(l, m) : -0.5 * ladder_A(l - 1, m - 1);
}

}  // namespace

std::vector<CouplingRow> closure_pn(int N) {
  // Real rows obtained by applying the unitary change of variables to the
  // complex rows (written out by hand; R_l^m = ((-1)^m psi^m + psi^-m)/sqrt2,
  // I_l^m = i((-1)^m psi^m - psi^-m)/sqrt2, R_l^0 = psi^0):
  //   M_x: R_l^0 -> R^1: -sqrt2 a+;  R_l^m -> R^{m+1}: -a+,  R^{m-1}: -k_m a-;
  //        I_l^m -> I^{m+1}: -a+,  I^{m-1} (m >= 2): -a-
  //   M_y: R_l^0 -> I^1: -sqrt2 a+;  R_l^m -> I^{m+1}: -a+,  I^{m-1} (m >= 2): +a-;
  //        I_l^m -> R^{m+1}: +a+,  R^{m-1}: -k_m a-
  // with a+- = alpha_plus/minus(l, l', m), l' = l -+ 1, k_1 = sqrt2, k_m = 1 else.
  const auto moms = moment_list(N);
  std::map<std::tuple<int, int, int>, int> index;  // (imag, l, m) -> k
  for (size_t k = 0; k < moms.size(); ++k) index[{moms[k].imag, moms[k].l, moms[k].m}] = int(k);
  auto find = [&](int imag, int l, int m) -> int {
    if (l < 0 || l > N || m < 0 || m > l) return -1;
    if (imag && m == 0) return -1;
    auto it = index.find({imag, l, m});
    return it == index.end() ? -1 : it->second;
  };
  const double s2 = std::sqrt(2.0);
  std::vector<CouplingRow> rows(moms.size());
  for (size_t k = 0; k < moms.size(); ++k) {
    const int im = moms[k].imag, l = moms[k].l, m = moms[k].m;
    CouplingRow& r = rows[k];
    auto add = [&](bool is_x, int imag, int lp, int mp, double v) {
      int col = find(imag, lp, mp);
      if (col < 0 || v == 0.0) return;
      if (is_x) {
        if (r.nx >= 4) throw std::runtime_error("more than four x couplings");
        r.x[r.nx++] = {col, v};
      } else {
        if (r.ny >= 4) throw std::runtime_error("more than four y couplings");
        r.y[r.ny++] = {col, v};
      }
    };
    for (int lp : {l - 1, l + 1}) {
      if (lp < 0 || lp > N) continue;
      const double ap = alpha_plus(l, lp, m);
      const double am = alpha_minus(l, lp, m);
      const double km = (m == 1) ? s2 : 1.0;
      if (m == 0) {
        // the I_l^0 component does not exist: R_l^0 is the only m = 0 row
        add(true, 0, lp, 1, -s2 * ap);
        add(false, 1, lp, 1, -s2 * ap);
      } else if (!im) {
        add(true, 0, lp, m + 1, -ap);
        add(true, 0, lp, m - 1, -km * am);
        add(false, 1, lp, m + 1, -ap);
        if (m >= 2) add(false, 1, lp, m - 1, am);
      } else {
        add(true, 1, lp, m + 1, -ap);
        if (m >= 2) add(true, 1, lp, m - 1, -am);
        add(false, 0, lp, m + 1, ap);
        add(false, 0, lp, m - 1, -km * am);
      }
    }
  }
  return rows;
}

namespace {

// Number of eigenvalues of the symmetric tridiagonal (alpha, beta) below x
// (Sturm sequence count).
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i ? bb / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++cnt;
  }
  return cnt;
}

}  // namespace

double spectral_radius_x(const std::vector<CouplingRow>& rows) {
  const int n = int(rows.size());
  if (n == 1) return 0.0;
  auto matvec = [&](const std::vector<double>& v, std::vector<double>& w) {
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int t = 0; t < rows[i].nx; ++t) s += rows[i].x[t].val * v[rows[i].x[t].col];
      w[i] = s;
    }
  };
  const int kmax = std::min(n, 400);
  std::vector<std::vector<double>> V;
  std::vector<double> alpha, beta;
  std::vector<double> v(n), w(n);
  uint64_t seed = 0x9E3779B97F4A7C15ull;
  auto fresh = [&](std::vector<double>& x) {
    for (int i = 0; i < n; ++i) {
      seed = seed * 6364136223846793005ull + 1442695040888963407ull;
      x[i] = double((seed >> 11) & 0xFFFFF) / double(0xFFFFF) + 0.5;
    }
  };
  auto orthonormalise = [&](std::vector<double>& x) -> double {
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& q : V) {
        double d = 0.0;
        for (int i = 0; i < n; ++i) d += q[i] * x[i];
        for (int i = 0; i < n; ++i) x[i] -= d * q[i];
      }
    double nr = 0.0;
    for (int i = 0; i < n; ++i) nr += x[i] * x[i];
    nr = std::sqrt(nr);
    if (nr > 0) for (int i = 0; i < n; ++i) x[i] /= nr;
    return nr;
  };
  fresh(v);
  orthonormalise(v);
  double b_prev = 0.0;
  for (int k = 0; k < kmax; ++k) {
    V.push_back(v);
    matvec(v, w);
    double a = 0.0;
    for (int i = 0; i < n; ++i) a += v[i] * w[i];
    alpha.push_back(a);
    if (k + 1 == kmax) break;
    double nr = orthonormalise(w);
    if (nr < 1e-10) {
      // invariant subspace: continue in its orthogonal complement with beta = 0
      fresh(w);
      nr = orthonormalise(w);
      if (nr < 1e-10) break;
      beta.push_back(0.0);
    } else {
      beta.push_back(nr);
    }
    v = w;
    (void)b_prev;
  }
  beta.resize(alpha.size() > 0 ? alpha.size() - 1 : 0);
  double bound = 0.0;
  for (size_t i = 0; i < alpha.size(); ++i) {
    double r = std::fabs(alpha[i]) + (i ? std::fabs(beta[i - 1]) : 0.0) +
               (i + 1 < alpha.size() ? std::fabs(beta[i]) : 0.0);
    bound = std::max(bound, r);
  }
  const int m = int(alpha.size());
  // largest eigenvalue: smallest x with count(x) == m
  double lo = -bound - 1.0, hi = bound + 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(alpha, beta, mid) >= m) hi = mid; else lo = mid;
  }
  const double lmax = hi;
  lo = -bound - 1.0;
  hi = bound + 1.0;
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sturm_count(alpha, beta, mid) >= 1) hi = mid; else lo = mid;
  }
  const double lmin = lo;
  return std::max(std::fabs(lmax), std::fabs(lmin));
}

void time_step(double cfl, double dx, double dy, double rho, double t_final, double* dt,
               int64_t* nsteps) {
  // Thm. 1 (dt < h for P_1), scaled by 1/rho(M) and by the 2D factor carried in
  // cfl (Sect. 4.6); the step count is rounded up so the run lands on t_final.
  double dt0 = cfl * std::min(dx, dy) / rho;
  int64_t n = (int64_t)std::ceil(t_final / dt0 - 1e-12);
  if (n < 1) n = 1;
  *nsteps = n;
  *dt = t_final / double(n);
}

DecayMap decay_map(int N, bool anisotropic) {
  const auto moms = moment_list(N);
  DecayMap dm;
  dm.dk.assign(moms.size(), -1);
  std::map<std::tuple<int, int, int>, int> planes;
  auto plane = [&](int gx, int gy, int l) {
    auto key = std::make_tuple(gx, gy, l);
    auto it = planes.find(key);
    if (it != planes.end()) return it->second;
    int id = dm.nplanes++;
    planes[key] = id;
    dm.plane_gx.push_back(gx);
    dm.plane_gy.push_back(gy);
    dm.plane_l.push_back(l);
    return id;
  };
  for (size_t k = 0; k < moms.size(); ++k) {
    const auto& mi = moms[k];
    int l = (k == 0) ? -1 : (anisotropic ? mi.l : 1);
    dm.dk[k] = plane(mi.gx, mi.gy, l);
  }
  return dm;
}

SweepProgram build_sweep_program(int N, int parity, int tx, int ty, double dx, double dy,
                                 const std::vector<CouplingRow>& rows, const DecayMap& dm,
                                 const std::vector<int32_t>& qk) {
  // Outputs of order l (l of the sweep's parity) need the other-parity orders
  // l-1 and l+1; orders are visited ascending and the staged planes of order
  // l+1 are kept for the next output order.  Two LDS buffers of N+1 planes,
  // selected by bit 1 of the input order, hold the window.
  const auto moms = moment_list(N);
  SweepProgram p;
  p.parity = parity;
  p.tx = tx;
  p.ty = ty;
  const int B = N + 1;
  const int nmom = int(moms.size());
  // two order buffers, one plane of zeros that the padding terms read, and the
  // source tiles of this sweep's outputs (staged once, before the first order)
  std::vector<int> src_slot(nmom, -1);
  int nsrc_used = 0;
  for (int k = 0; k < nmom; ++k) {
    const bool even = moms[k].gx == moms[k].gy;
    if (!qk.empty() && qk[k] >= 0 && (parity == 0) == even) src_slot[k] = 2 * B + 1 + nsrc_used++;
  }
  p.slots = 2 * B + 1 + nsrc_used;
  const int zero_off = 2 * B * (tx + 1) * (ty + 1);
  p.zero_off = zero_off;
  const int LW = tx + 1;
  const int P = (tx + 1) * (ty + 1);
  std::vector<int> pos_in_order(moms.size(), 0);
  {
    std::vector<int> cnt(N + 2, 0);
    for (size_t k = 0; k < moms.size(); ++k) pos_in_order[k] = cnt[moms[k].l]++;
  }
  auto lds_of = [&](int k) { return (((moms[k].l >> 1) & 1) * B + pos_in_order[k]) * P; };
  for (int l = parity; l <= N; l += 2) {
    SweepOrder o;
    o.load0 = int(p.loads.size());
    for (int lin : {l - 1, l + 1}) {
      if (lin < 0 || lin > N) continue;
      if (lin == l - 1 && l != parity) continue;  // already staged by the previous order
      for (size_t k = 0; k < moms.size(); ++k) {
        if (moms[k].l != lin) continue;
        SweepLoad ld;
        ld.k = int(k);
        ld.lds = lds_of(int(k));
        ld.ox = moms[k].gx == AXIS_CELL ? 1 : 0;
        ld.oy = moms[k].gy == AXIS_CELL ? 1 : 0;
        p.loads.push_back(ld);
      }
    }
    if (l == parity) {
      for (int k = 0; k < nmom; ++k) {
        if (src_slot[k] < 0) continue;
        // a source tile is read at the output point itself: no halo offset
        p.loads.push_back({nmom + qk[k], src_slot[k] * (tx + 1) * (ty + 1), 0, 0});
      }
    }
    o.load1 = int(p.loads.size());
    p.max_loads = std::max(p.max_loads, o.load1 - o.load0);
    o.row0 = int(p.rows.size());
    for (size_t k = 0; k < moms.size(); ++k) {
      if (moms[k].l != l) continue;
      const auto& mk = moms[k];
      SweepRow row;
      row.k = int(k);
      // output grids of the sweep: even -> G11 (slot 0), G22 (slot 1);
      // odd -> G21 (slot 0), G12 (slot 1)
      row.gslot = (mk.gx == mk.gy) ? (mk.gx == AXIS_CELL ? 0 : 1) : (mk.gx == AXIS_NODE ? 0 : 1);
      row.dk = dm.dk[k];
      row.so = src_slot[k] >= 0 ? src_slot[k] * (tx + 1) * (ty + 1) : -1;
      const CouplingRow& r = rows[k];
      double cf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int t = 0; t < 4; ++t) {
        row.xo[t] = zero_off;
        row.yo[t] = zero_off;
      }
      for (int t = 0; t < r.nx; ++t) {
        const int j = r.x[t].col;
        const int oy = moms[j].gy == AXIS_CELL ? 1 : 0;
        // D_x at output (tx, ty): L[ty+oy][tx+1] - L[ty+oy][tx]
        row.xo[t] = lds_of(j) + oy * LW;
        cf[t] = -r.x[t].val / dx;
      }
      for (int t = 0; t < r.ny; ++t) {
        const int j = r.y[t].col;
        const int ox = moms[j].gx == AXIS_CELL ? 1 : 0;
        // D_y at output (tx, ty): L[ty+1][tx+ox] - L[ty][tx+ox]
        row.yo[t] = lds_of(j) + ox;
        cf[4 + t] = -r.y[t].val / dy;
      }
      row.nx = r.nx;
      row.ny = r.ny;
      p.rows.push_back(row);
      p.coefs.insert(p.coefs.end(), cf, cf + 8);
    }
    o.row1 = int(p.rows.size());
    p.max_rows = std::max(p.max_rows, o.row1 - o.row0);
    p.orders.push_back(o);
  }
  return p;
}

}  // namespace starmap
