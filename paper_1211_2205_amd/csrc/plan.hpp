// Host plan of the staggered-grid P_N step: moments, moment matrices, grid
// classes, spectral radius, time step, and the per-parity sweep programs that
// drive the device kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace starmap {

// Grid type along one axis: cell centres or nodes.
enum AxisType : int { AXIS_CELL = 1, AXIS_NODE = 2 };

struct MomentInfo {
  int imag;  // 0: R_l^m, 1: I_l^m
  int l, m;
  int gx, gy;  // grid G_{gx gy}: 1 = cell centres, 2 = nodes along that axis
};

// Real moments in the order R_0^0, R_1^1, I_1^1, R_2^2, I_2^2, R_2^0, ...
// (order l ascending, m descending, R before I).
std::vector<MomentInfo> moment_list(int N);
int moment_count(int N);

struct Coupling {
  int col;
  double val;
};
struct CouplingRow {
  int nx = 0, ny = 0;
  Coupling x[4];
  Coupling y[4];
};

// Rows of the real moment matrices M_x, M_y (at most four nonzeros each).
std::vector<CouplingRow> closure_pn(int N);

// Largest eigenvalue magnitude of M_x (Lanczos with full reorthogonalisation
// plus Sturm bisection on the tridiagonal matrix).
double spectral_radius_x(const std::vector<CouplingRow>& rows);

// Time step rule: dt0 = cfl * min(dx, dy) / rho; n = ceil(t_final / dt0);
// dt = t_final / n.
void time_step(double cfl, double dx, double dy, double rho, double t_final, double* dt,
               int64_t* nsteps);

// One order-window of a parity sweep: planes of the other parity to stage in
// LDS, then the output rows to update.
struct SweepLoad {
  int32_t k;       // input plane (moment index)
  int32_t lds;     // element offset of its LDS tile
  int32_t ox, oy;  // 1 if the input is cell-centred along x / y (halo on the low side)
};
// One output row of a sweep: the moment it updates and its (at most) four
// x- and four y-couplings, padded with zero couplings that read the zero plane.
struct SweepRow {
  int32_t k;      // output plane (moment index)
  int32_t gslot;  // which of the sweep's two output grids (decay cache slot)
  int32_t dk;     // decay plane index
  int32_t so;     // LDS element offset of the staged source tile, or -1
  int32_t xo[4];  // LDS element offset of the lower sample of each x difference
  int32_t yo[4];  // LDS element offset of the lower sample of each y difference
  int32_t nx, ny; // real couplings among the four of each kind
};
struct SweepOrder {
  int32_t load0, load1, row0, row1;
};

struct SweepChunk {
  int32_t order0, order1;  // output orders of one m range
};

struct SweepProgram {
  int parity = 0;  // outputs: 0 = even components (G11, G22), 1 = odd (G21, G12)
  int tx = 0, ty = 0;
  int nchunks = 1;       // m ranges; each tile is processed by nchunks workgroups
  int buffer_planes = 0; // planes per order buffer
  int slots = 0;         // LDS planes: two order buffers, the zero plane, source tiles
  int zero_off = 0;      // LDS element offset of the zero plane
  std::vector<SweepChunk> chunks;
  int max_rows = 0;  // most output rows of one order
  int max_loads = 0; // most planes staged for one order
  std::vector<SweepOrder> orders;
  std::vector<SweepLoad> loads;
  std::vector<SweepRow> rows;
  // eight coefficients per row: x couplings then y couplings, pre-scaled by
  // -1/dx and -1/dy so that W = sum coef * (upper - lower sample)
  std::vector<double> coefs;
  // host-side record of the input plane behind each coupling (-1 for padding),
  // eight per row, for validate_sweep_program
  std::vector<int32_t> coupled;
};

// Replays a program's LDS slot contents and checks that every coupling and
// source read finds the plane it expects; returns an empty string or a message.
std::string validate_sweep_program(int N, const SweepProgram& p, const std::vector<CouplingRow>& rows,
                                   const std::vector<int32_t>& qk);

struct DecayMap {
  std::vector<int32_t> dk;  // per moment: decay plane index
  int nplanes = 0;
  // plane p describes (grid gx, gy, order l); l = -1 for the absorption-only
  // plane of the zeroth moment
  std::vector<int32_t> plane_gx, plane_gy, plane_l;
};

// Decay planes: the zeroth moment decays with sigma_a; moments of order l >= 1
// with sigma_a + sigma_s0 - sigma_sl.  Isotropic scattering shares one plane
// per grid for all l >= 1.
DecayMap decay_map(int N, bool anisotropic);

// Moments of a unit beam delta(Omega - Omega_0) (the real basis functions at
// Omega_0), in moment order.
std::vector<double> direction_moments(int N, double ox, double oy, double oz);

// Number of m ranges of the given width for order N.
int sweep_chunk_count(int N, int width);

// qk[k] >= 0 marks moment k as carrying source plane qk[k]; source planes are
// stored after the nmom state planes (plane index nmom + qk[k]).
SweepProgram build_sweep_program(int N, int parity, int tx, int ty, double dx, double dy,
                                 const std::vector<CouplingRow>& rows, const DecayMap& dm,
                                 const std::vector<int32_t>& qk, int nchunks);

}  // namespace starmap
