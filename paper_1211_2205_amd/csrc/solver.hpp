// Private interface of the library's host side: the solver object and the
// helpers shared by the C-ABI sources (capi.cpp, closure.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/starmap.h"
#include "kernels.hpp"
#include "mlp.hpp"
#include "plan.hpp"

namespace starmap {
namespace detail {

// Records msg as the calling thread's last error and returns code.
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return fail(STARMAP_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));     \
  } while (0)

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct FieldTerm {
  starmap_field_fn space = nullptr;
  void* space_ctx = nullptr;
  starmap_time_fn time = nullptr;
  void* time_ctx = nullptr;
};

struct FieldSource {
  starmap_field_fn fn = nullptr;
  void* ctx = nullptr;
  bool time_dependent = false;
  // pre-sampled values on grid g = (gx-1) + 2 (gy-1), public layout
  std::array<std::vector<double>, 4> arrays;
  bool has_array[4] = {false, false, false, false};
  // separable form sum a_i(t) g_i(x, y) (used instead of fn / arrays when non-empty)
  std::vector<FieldTerm> terms;
  bool set() const {
    return fn || has_array[0] || has_array[1] || has_array[2] || has_array[3] || !terms.empty();
  }
};


inline int grid_id(int gx, int gy) { return (gx - 1) + 2 * (gy - 1); }

}  // namespace detail
}  // namespace starmap

struct starmap_solver {
  starmap_problem prob{};
  int N = 0, nmom = 0;
  std::vector<starmap::MomentInfo> moms;
  std::vector<starmap::CouplingRow> rows;
  double rho = 0, dx = 0, dy = 0, dt = 0;
  int64_t steps_total = 0, steps_done = 0;
  double t = 0;
  int nx = 0, ny = 0, px = 0, py = 0;
  int storage = starmap::STORE_FP64;
  size_t ssize = 8, csize = 8;
  int pitch = 0, nrows = 0;
  int64_t plane_stride = 0;

  starmap::detail::FieldSource absorption, scattering;
  std::map<int, starmap::detail::FieldSource> scattering_order;  // l -> sigma_sl
  std::map<int, starmap::detail::FieldSource> source;            // k -> q_k
  std::map<int, starmap::detail::FieldSource> initial;           // k -> u_k(0)
  bool anisotropic = false;
  // filtered P_N: damping added to the decay of each order (empty: none)
  std::vector<double> damping;
  // diffusion-corrected P_N: kappa of the diffusion step on the order-N moments
  starmap::detail::FieldSource diffusion;
  bool has_diffusion = false;
  // parity-fused passes (small orders): second state buffer and the per-moment table
  bool fused = false, fused_ready = false;
  size_t off_state2 = 0, off_ftab = 0;
  std::vector<int32_t> ftab;   // 16 ints per moment, then the moment order (odd first)
  std::vector<double> fcoef;   // 8 coefficients per moment
  int fnodd = 0;
  size_t off_dtmp = 0, off_kappa = 0, off_dtab = 0;  // scratch planes, kappa planes, plane table
  bool diffusion_ready = false;
  bool time_dependent = false;

  starmap::DecayMap dmap;
  std::vector<int32_t> qk;  // per moment: source plane or -1
  int nsrc = 0;

  // device
  void* dev = nullptr;
  size_t dev_bytes = 0;
  bool owns_dev = false;
  bool owns_stream = false;
  hipStream_t stream = nullptr;
  bool bound = false;
  size_t off_state = 0, off_decay = 0, off_src = 0, off_prog[2] = {0, 0}, off_diag = 0;
  size_t prog_bytes[2] = {0, 0};
  int diag_rows_per_block = 64, diag_nblocks = 0;

  bool device_ready = false;     // workspace allocated and state uploaded
  bool materials_ready = false;  // decay and source planes uploaded for current time
  int variant = -1;              // -1: not chosen yet
  int slots = 0;
  int nchunks = 1;               // m ranges per tile (workgroups per tile and sweep)
  int chunk_width = 0;           // m indices per range (0: default)
  int tile_strip = 8;            // tile order of the sweep: strips of k tile rows (k >= 2) or -k columns (k <= -2)
  starmap::SweepProgram prog[2];
  bool prog_uploaded = false;

  // HIP graphs of runs of the repeated pair (S^e_dt, S^o_dt) of the plain
  // composition, one per power-of-two pair count; dropped whenever the launch
  // sequence may change (graph_version, bumped by upload_program)
  bool use_graphs = true;
  int graph_version = 0, pair_graphs_version = -1;
  std::map<int, hipGraphExec_t> pair_graphs;

  // per-launch HIP events of the sweep kernel (starmap_profile_begin/end)
  bool profiling = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double prof_bytes = 0.0;
  double sweep_bytes_cache[2] = {-1.0, -1.0};

  // learned closure (order 5): network region, geometry, weights loaded
  bool closure = false;
  bool closure_loaded = false;
  // fused closure sweep (starmap_closure_set_fused; batches always use it):
  // the order-5 moments alternate between their state planes (A) and the
  // closure planes (B); c5_flip = 1 while the current values sit in B (only
  // between the odd sweeps of one advance call); the even sweep then reads
  // them through a second program (off_prog_b)
  bool closure_fused = false;
  int c5_flip = 0;
  size_t off_prog_b = 0;
  starmap::ClosureOdd codd{};
  std::vector<float> closure_w;  // the loaded parameter blob (batches need one network)
  size_t off_net = 0;
  starmap::ClosureGeo cgeo{};
  void* sample_buf = nullptr;  // device copy of training-sample points
  size_t sample_cap = 0;

  // time-separable fields on the device: basis planes (compute type) and an
  // int32 table: per output (every decay plane, then every source plane) the
  // first of its entries; per entry (basis plane, time factor or -1, sign);
  // four lists of (output, destination plane) pairs: all decay outputs, decay
  // outputs with a time factor, all source outputs, source outputs with one.
  bool separable = false;
  size_t off_basis = 0, off_comb = 0;
  int nbasis = 0;
  struct Basis {
    const starmap::detail::FieldSource* field;
    int term;  // -1: the whole (time-independent) field
    int gx, gy;
  };
  std::vector<Basis> basis;
  std::vector<starmap::detail::FieldTerm> time_terms;
  std::vector<int32_t> comb_tab;
  std::vector<double> comb_cst;  // per output: constant term (filter damping of decay planes)
  int tab_first = 0, tab_entries = 0, tab_list[4] = {}, nlist[4] = {};
  bool basis_ready = false, static_done = false;

  // plane_stride is a multiple of 128 elements, so planes of every element
  // size start 256-byte aligned and state and material planes share one
  // element stride
  size_t plane_bytes_state() const { return size_t(plane_stride) * ssize; }
  size_t plane_bytes_c() const { return size_t(plane_stride) * csize; }
};

namespace starmap {
namespace detail {

int points_x(const starmap_solver* s, int gx);
int points_y(const starmap_solver* s, int gy);
char* dptr(const starmap_solver* s, size_t off);
int ensure_device(starmap_solver* s);
int upload_materials(starmap_solver* s, double t_eval);
// Materials of a time-independent or separable problem at t_eval.
int ensure_materials(starmap_solver* s, double t_eval);
// Largest dynamic LDS of one workgroup on the current device (64 KiB without one).
int max_lds_bytes();

// Closure (closure.cpp): geometry of a solver's closure inputs, and the
// fused closure kernel run before every odd sweep of a closure solver.
int closure_geometry(const starmap_solver* s, ClosureGeo* g, bool with_terms);
int closure_before_odd(starmap_solver* s);
// Fused closure solvers: the odd sweep with the network (flips c5_flip), and
// the copy that puts the order-5 moments back into their state planes.
int closure_odd_sweep(starmap_solver* s, double tau);
int closure_settle(starmap_solver* s);
// First plane of the order-5 moments in A (state) and in B (closure planes).
int closure_plane_a(const starmap_solver* s);
int closure_plane_b(const starmap_solver* s);

}  // namespace detail
}  // namespace starmap
