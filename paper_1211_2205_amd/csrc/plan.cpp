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
  // cfl (Sect. 4.5); the step count is rounded up so the run lands on t_final.
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

int sweep_chunk_count(int N, int width) {
  if (width < 2) width = 2;
  int k = (N + 1 + width - 1) / width;
  // every range must hold both parities of m so that no order inside a
  // chunk's span is empty
  return std::max(1, std::min(k, (N + 1) / 2));
}

SweepProgram build_sweep_program(int N, int parity, int tx, int ty, double dx, double dy,
                                 const std::vector<CouplingRow>& rows, const DecayMap& dm,
                                 const std::vector<int32_t>& qk, int nchunks) {
  // The outputs of one parity are split into nchunks ranges of the azimuthal
  // index m.  A chunk's output (l, m) couples to the other parity at orders
  // l -+ 1 and indices m -+ 1 only (Lemma 2), so the chunk needs the inputs
  // with m' in [m0 - 1, m1].  Within a chunk, output orders are visited
  // descending; the window holds the input orders l + 1 and l - 1, and the
  // planes of l - 1 stay staged for output order l - 2.  Two LDS buffers of B
  // planes (selected by bit 1 of the input order), a plane of zeros for the
  // padding couplings, and the source tiles of one order's rows (staged with
  // that order's planes) make up the LDS.
  const auto moms = moment_list(N);
  const int nmom = int(moms.size());
  SweepProgram p;
  p.parity = parity;
  p.tx = tx;
  p.ty = ty;
  nchunks = std::max(1, std::min(nchunks, (N + 1) / 2));
  p.nchunks = nchunks;
  const int LW = tx + 1;
  const int P = (tx + 1) * (ty + 1);
  auto is_out = [&](int k) { return (parity == 0) == (moms[k].gx == moms[k].gy); };
  // m ranges of equal width
  std::vector<int> mlo(nchunks), mhi(nchunks);
  for (int c = 0; c < nchunks; ++c) {
    mlo[c] = (N + 1) * c / nchunks;
    mhi[c] = (N + 1) * (c + 1) / nchunks;
  }
  auto in_window = [&](int c, int k) { return moms[k].m >= mlo[c] - 1 && moms[k].m <= mhi[c]; };
  // buffer size: most input planes of one order inside one chunk's window
  int B = 1;
  for (int c = 0; c < nchunks; ++c) {
    std::vector<int> cnt(N + 2, 0);
    for (int k = 0; k < nmom; ++k)
      if (!is_out(k) && in_window(c, k)) B = std::max(B, ++cnt[moms[k].l]);
  }
  // source tiles are staged with their order's planes: slots for the most
  // rows with a source in one order of one chunk
  auto has_src = [&](int k) { return !qk.empty() && qk[k] >= 0; };
  int max_src = 0;
  for (int c = 0; c < nchunks; ++c)
    for (int l = 0; l <= N; ++l) {
      int n = 0;
      for (int k = 0; k < nmom; ++k)
        if (moms[k].l == l && is_out(k) && has_src(k) && moms[k].m >= mlo[c] && moms[k].m < mhi[c]) ++n;
      max_src = std::max(max_src, n);
    }
  p.slots = 2 * B + 1 + max_src;
  const int zero_off = 2 * B * P;
  p.zero_off = zero_off;
  p.buffer_planes = B;

  for (int c = 0; c < nchunks; ++c) {
    SweepChunk ch;
    ch.order0 = int(p.orders.size());
    // positions of the chunk's input planes within their order
    std::vector<int> pos(nmom, -1);
    {
      std::vector<int> cnt(N + 2, 0);
      for (int k = 0; k < nmom; ++k)
        if (!is_out(k) && in_window(c, k)) pos[k] = cnt[moms[k].l]++;
    }
    auto lds_of = [&](int k) { return (((moms[k].l >> 1) & 1) * B + pos[k]) * P; };
    // source tile slot of each row with a source: its rank among the rows of
    // its order that have one
    std::vector<int> src_off(nmom, -1);
    for (int l = 0; l <= N; ++l) {
      int n = 0;
      for (int k = 0; k < nmom; ++k)
        if (moms[k].l == l && is_out(k) && has_src(k) && moms[k].m >= mlo[c] && moms[k].m < mhi[c])
          src_off[k] = (2 * B + 1 + n++) * P;
    }
    // Orders are visited from the top down: every chunk of a tile starts at
    // the highest order at the same time, so the input planes that two
    // neighbouring m ranges share are requested together (one HBM read, the
    // second from L2).
    bool first = true;
    const int top = ((N - parity) % 2 == 0) ? N : N - 1;
    for (int l = top; l >= parity; l -= 2) {
      // output rows of this order inside the chunk
      std::vector<int> outs;
      for (int k = 0; k < nmom; ++k)
        if (moms[k].l == l && is_out(k) && moms[k].m >= mlo[c] && moms[k].m < mhi[c]) outs.push_back(k);
      if (outs.empty()) {
        // m <= l: below the chunk's lowest order no rows exist, and with two
        // or more m values per range no order inside the span is empty
        if (first) throw std::runtime_error("sweep chunk without rows at the top order");
        break;
      }
      SweepOrder o;
      o.load0 = int(p.loads.size());
      for (int lin : {l + 1, l - 1}) {
        if (lin < 0 || lin > N) continue;
        if (lin == l + 1 && !first) continue;  // staged by the previous (higher) order
        for (int k = 0; k < nmom; ++k) {
          if (moms[k].l != lin || pos[k] < 0) continue;
          SweepLoad ld;
          ld.k = k;
          ld.lds = lds_of(k);
          ld.ox = moms[k].gx == AXIS_CELL ? 1 : 0;
          ld.oy = moms[k].gy == AXIS_CELL ? 1 : 0;
          p.loads.push_back(ld);
        }
      }
      for (int k : outs) {
        if (src_off[k] < 0) continue;
        // a source tile is read at the output point itself: no halo offset
        p.loads.push_back({nmom + qk[k], src_off[k], 0, 0});
      }
      first = false;
      o.load1 = int(p.loads.size());
      p.max_loads = std::max(p.max_loads, o.load1 - o.load0);
      o.row0 = int(p.rows.size());
      for (int k : outs) {
        const auto& mk = moms[k];
        SweepRow row;
        row.k = k;
        // output grids of the sweep: even -> G11 (slot 0), G22 (slot 1);
        // odd -> G21 (slot 0), G12 (slot 1)
        row.gslot = (mk.gx == mk.gy) ? (mk.gx == AXIS_CELL ? 0 : 1) : (mk.gx == AXIS_NODE ? 0 : 1);
        row.dk = dm.dk[k];
        row.so = src_off[k];
        const CouplingRow& r = rows[k];
        double cf[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int32_t coupled[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
        for (int t = 0; t < 4; ++t) {
          row.xo[t] = zero_off;
          row.yo[t] = zero_off;
        }
        for (int t = 0; t < r.nx; ++t) {
          const int j = r.x[t].col;
          if (pos[j] < 0) throw std::runtime_error("coupling outside the chunk window");
          const int oy = moms[j].gy == AXIS_CELL ? 1 : 0;
          // D_x at output (tx, ty): L[ty+oy][tx+1] - L[ty+oy][tx]
          row.xo[t] = lds_of(j) + oy * LW;
          cf[t] = -r.x[t].val / dx;
          coupled[t] = j;
        }
        for (int t = 0; t < r.ny; ++t) {
          const int j = r.y[t].col;
          if (pos[j] < 0) throw std::runtime_error("coupling outside the chunk window");
          const int ox = moms[j].gx == AXIS_CELL ? 1 : 0;
          // D_y at output (tx, ty): L[ty+1][tx+ox] - L[ty][tx+ox]
          row.yo[t] = lds_of(j) + ox;
          cf[4 + t] = -r.y[t].val / dy;
          coupled[4 + t] = j;
        }
        row.nx = r.nx;
        row.ny = r.ny;
        p.rows.push_back(row);
        p.coefs.insert(p.coefs.end(), cf, cf + 8);
        p.coupled.insert(p.coupled.end(), coupled, coupled + 8);
      }
      o.row1 = int(p.rows.size());
      p.max_rows = std::max(p.max_rows, o.row1 - o.row0);
      p.orders.push_back(o);
    }
    ch.order1 = int(p.orders.size());
    p.chunks.push_back(ch);
  }
  return p;
}

std::string validate_sweep_program(int N, const SweepProgram& p, const std::vector<CouplingRow>& rows,
                                   const std::vector<int32_t>& qk) {
  const auto moms = moment_list(N);
  const int nmom = int(moms.size());
  const int LW = p.tx + 1;
  const int P = (p.tx + 1) * (p.ty + 1);
  auto msg = [](const std::string& m) { return m; };
  if (p.zero_off != 2 * p.buffer_planes * P) return msg("zero plane offset");
  std::vector<int> seen(nmom, 0);
  for (size_t c = 0; c < p.chunks.size(); ++c) {
    std::vector<int> slot(p.slots, -1);
    for (int o = p.chunks[c].order0; o < p.chunks[c].order1; ++o) {
      const SweepOrder& ord = p.orders[o];
      for (int i = ord.load0; i < ord.load1; ++i) {
        const SweepLoad& ld = p.loads[i];
        if (ld.lds % P || ld.lds / P >= p.slots || ld.lds == p.zero_off) return msg("load slot out of range");
        slot[ld.lds / P] = ld.k;
      }
      for (int r = ord.row0; r < ord.row1; ++r) {
        const SweepRow& row = p.rows[r];
        const int k = row.k;
        if (++seen[k] > 1) return msg("moment updated twice in one sweep");
        if ((p.parity == 0) != (moms[k].gx == moms[k].gy)) return msg("row of the wrong parity");
        for (int t = 0; t < 8; ++t) {
          const int off = t < 4 ? row.xo[t] : row.yo[t - 4];
          const int j = p.coupled[8 * r + t];
          if (j < 0) {
            if (off != p.zero_off || p.coefs[8 * r + t] != 0.0) return msg("padding coupling");
            continue;
          }
          const int s = off / P, sub = off % P;
          if (s >= p.slots || slot[s] != j) return msg("coupling reads a plane that is not staged");
          const bool x = t < 4;
          const int want = x ? (moms[j].gy == AXIS_CELL ? LW : 0) : (moms[j].gx == AXIS_CELL ? 1 : 0);
          if (sub != want) return msg("coupling halo offset");
          // the coupling is a real matrix entry of this row
          const CouplingRow& cr = rows[k];
          bool found = false;
          const int n = x ? cr.nx : cr.ny;
          for (int u = 0; u < n; ++u)
            if ((x ? cr.x[u].col : cr.y[u].col) == j) found = true;
          if (!found) return msg("coupling not in the moment matrix");
        }
        if (row.so >= 0) {
          if (row.so % P || slot[row.so / P] != nmom + qk[k]) return msg("source tile not staged");
        } else if (!qk.empty() && qk[k] >= 0) {
          return msg("source of a row dropped");
        }
      }
    }
  }
  for (int k = 0; k < nmom; ++k) {
    const bool out = (p.parity == 0) == (moms[k].gx == moms[k].gy);
    if (out && seen[k] != 1) return msg("moment not updated by its sweep");
    // every real coupling of an updated row is present
    if (out) {
      int cnt = 0;
      for (size_t r = 0; r < p.rows.size(); ++r)
        if (p.rows[r].k == k)
          for (int t = 0; t < 8; ++t) cnt += p.coupled[8 * r + t] >= 0;
      if (cnt != rows[k].nx + rows[k].ny) return msg("coupling dropped");
    }
  }
  return std::string();
}

std::vector<double> direction_moments(int N, double ox, double oy, double oz) {
  // Real orthonormal basis at Omega = (ox, oy, oz): with mu = oz, s = sqrt(1 - mu^2)
  // and the azimuth phi of (ox, oy), R_l^0 = Pbar_l^0(mu), R_l^m = sqrt2 Pbar_l^m(mu)
  // cos(m phi), I_l^m = sqrt2 Pbar_l^m(mu) sin(m phi), where Pbar_l^m is the
  // associated Legendre function scaled to unit norm on the sphere,
  // sqrt((2l+1)/(4pi) (l-m)!/(l+m)!) P_l^m, by the stable three-term recurrences
  //   Pbar_m^m = sqrt((2m+1)/(2m)) s Pbar_{m-1}^{m-1},  Pbar_0^0 = 1/sqrt(4pi),
  //   Pbar_{m+1}^m = sqrt(2m+3) mu Pbar_m^m,
  //   Pbar_l^m = sqrt((4l^2-1)/(l^2-m^2)) (mu Pbar_{l-1}^m - sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)) Pbar_{l-2}^m).
  const double mu = oz, sn = std::sqrt(std::max(0.0, 1.0 - mu * mu));
  const double phi = std::atan2(oy, ox);
  std::vector<std::vector<double>> P(N + 1, std::vector<double>(N + 1, 0.0));
  double pmm = 1.0 / std::sqrt(4.0 * M_PI);
  for (int m = 0; m <= N; ++m) {
    if (m > 0) pmm *= std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * sn;
    P[m][m] = pmm;
    if (m + 1 <= N) P[m + 1][m] = std::sqrt(2.0 * m + 3.0) * mu * pmm;
    for (int l = m + 2; l <= N; ++l) {
      const double a = std::sqrt((4.0 * l * l - 1.0) / (double(l) * l - double(m) * m));
      const double b = std::sqrt((double(l - 1) * (l - 1) - double(m) * m) / (4.0 * (l - 1) * (l - 1) - 1.0));
      P[l][m] = a * (mu * P[l - 1][m] - b * P[l - 2][m]);
    }
  }
  std::vector<double> out;
  for (const MomentInfo& mi : moment_list(N)) {
    if (mi.m == 0)
      out.push_back(P[mi.l][0]);
    else
      out.push_back(std::sqrt(2.0) * P[mi.l][mi.m] * (mi.imag ? std::sin(mi.m * phi) : std::cos(mi.m * phi)));
  }
  return out;
}

}  // namespace starmap
