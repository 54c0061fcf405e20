/*
 * Oracle: plain FP64 CPU implementation of the StaRMAP half-step operators.
 *
 * TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU
 * baseline load this library.  It shares no code with the GPU library.
 *
 * Follows Seibold & Frank (arXiv 1211.2205), Sect. 4:
 *   - grids G11, G21, G12, G22 (eq. grid11, eq. staggered_grids) in the paper's
 *     index ranges: cell index i = 1..n at (i - 1/2) h, node index i = p..n at
 *     i h, stored from array position 0 upwards, x fastest;
 *   - half-grid central differences D_x, D_y (eq. central_differences);
 *   - boundary extension (Sect. 4.2): periodic wrap or constant extrapolation
 *     onto ghost points, applied before differencing;
 *   - residual r = q - M_x D_x u - M_y D_y u of the frozen other parity
 *     (eq. hyperbolic_balance_law_decoupled) and the exact sub-step solution
 *     u <- u + tau (r - c u) E(-c tau), E(z) = (e^z - 1)/z (eq. sub_step_solution).
 *
 * Plain loops; OpenMP only splits independent rows (one parallel region per
 * call), so results are identical for any thread count.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* number of grid points along an axis: type 1 = cell centres, 2 = nodes */
static int npts(int type, int n, int p) { return type == 1 ? n : n + 1 - p; }

/* E(z) = (exp(z) - 1) / z, E(0) = 1.
   mode 0: expm1(z) / z.
   mode 1: the paper's switch (Sect. 5.6): a three-term Taylor series below
           |z| <= 2e-4, else the plain quotient.  The series used is that of
           E itself, 1 + z/2 + z^2/6 (the printed series has the sign of the
           linear term flipped, i.e. it is the series of E(-z)). */
static double expm1div(double z, int mode) {
    if (z == 0.0) return 1.0;
    if (mode == 1) {
        if (fabs(z) <= 2e-4) return 1.0 + z / 2.0 + z * z / 6.0;
        return (exp(z) - 1.0) / z;
    }
    return expm1(z) / z;
}

double starmap_oracle_expm1div(double z, int mode) { return expm1div(z, mode); }

/* Thread count of the row loops (timing only: results do not depend on it). */
void starmap_oracle_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}
int starmap_oracle_threads(void) { return omp_get_max_threads(); }

/*
 * Boundary extension (Sect. 4.2) along one axis: the stored index of the
 * value at extended position a of a field of type `type` (1 = cell centres,
 * 2 = nodes) with n cells and periodicity flag p.  The difference onto the
 * other type at position a is (ext(a+1) - ext(a)) / h.
 *   type 1 (cells 1..n stored at 0..n-1, result on nodes p..n): extended
 *          cells p..n+1; ghost cell 0 := cell 1 (extrapolation; reached only
 *          when p = 0), ghost cell n+1 := cell n (extrapolation) or cell 1
 *          (periodic);
 *   type 2 (nodes p..n stored at 0..n-p, result on cells 1..n): extended
 *          nodes 0..n; node 0 := node n (periodic); extrapolation stores
 *          node 0 itself.
 */
static int ext_index(int type, int a, int n, int p) {
    if (type == 1) {
        int ci = p + a;              /* paper cell index, 0..n+1 */
        if (ci == 0) return 0;       /* ghost left := cell 1 */
        if (ci == n + 1) return p ? 0 : n - 1;
        return ci - 1;
    }
    if (a == 0 && p) return n - 1;   /* node 0 := node n */
    return a - p;
}

/* Row y of D_x: field on grid (tx, .) with rows of ns values -> nd values. */
static void diff_x_row(int tx, int nx, int px, double dx, const double* s, double* d) {
    const int nd = npts(3 - tx, nx, px);
    for (int a = 0; a < nd; ++a)
        d[a] = (s[ext_index(tx, a + 1, nx, px)] - s[ext_index(tx, a, nx, px)]) / dx;
}

/* Row a of D_y: field on grid (., ty) with `cols` values a row. */
static void diff_y_row(int ty, int ny, int py, double dy, int cols, const double* src, int a, double* d) {
    const double* hi = src + (size_t)ext_index(ty, a + 1, ny, py) * (size_t)cols;
    const double* lo = src + (size_t)ext_index(ty, a, ny, py) * (size_t)cols;
    for (int i = 0; i < cols; ++i) d[i] = (hi[i] - lo[i]) / dy;
}

static size_t plane_size(const int* gx, const int* gy, int k, int nx, int ny, int px, int py) {
    return (size_t)npts(gx[k], nx, px) * (size_t)npts(gy[k], ny, py);
}

/*
 * W_k = - sum_j Mx(k,j) D_x u_j - sum_j My(k,j) D_y u_j for every component k
 * of the given parity (even: G11 and G22; odd: G21 and G12).  Only the nonzero
 * entries of the rows are visited, j ascending, the x term before the y term.
 * W[k] must hold k's grid size for those k.  Returns 0, or -1 if a nonzero
 * entry couples grids that the staggering does not allow.
 *
 * One parallel region: first the differences of every component of the other
 * parity (rows split over threads), then every output row; each point's
 * arithmetic is the same for any thread count.
 */
int starmap_oracle_flux(int nx, int ny, int px, int py, double dx, double dy, int nmom,
                        const int* gx, const int* gy, const double* Mx, const double* My,
                        int parity, double* const* u, double* const* W) {
    if (nmom <= 0) return -1;
    /* the coupling pattern must match the staggering (checked up front) */
    for (int k = 0; k < nmom; ++k) {
        int even_k = gx[k] == gy[k];
        if ((parity == 0) != even_k) continue;
        for (int j = 0; j < nmom; ++j) {
            int other = (gx[j] == gy[j]) != even_k;
            if (Mx[(size_t)k * nmom + j] != 0.0 && (!other || 3 - gx[j] != gx[k] || gy[j] != gy[k])) return -1;
            if (My[(size_t)k * nmom + j] != 0.0 && (!other || gx[j] != gx[k] || 3 - gy[j] != gy[k])) return -1;
        }
    }
    double** DX = (double**)calloc((size_t)nmom, sizeof(double*));
    double** DY = (double**)calloc((size_t)nmom, sizeof(double*));
    for (int j = 0; j < nmom; ++j) {
        int even_j = gx[j] == gy[j];
        if ((parity == 0) == even_j) continue;  /* same parity as the outputs */
        DX[j] = (double*)malloc(sizeof(double) * (size_t)npts(3 - gx[j], nx, px) * (size_t)npts(gy[j], ny, py));
        DY[j] = (double*)malloc(sizeof(double) * (size_t)npts(gx[j], nx, px) * (size_t)npts(3 - gy[j], ny, py));
    }
#pragma omp parallel
    {
        for (int j = 0; j < nmom; ++j) {
            if (!DX[j]) continue;
            const int cols = npts(gx[j], nx, px), rows = npts(gy[j], ny, py);
            const int ndx = npts(3 - gx[j], nx, px), ndy = npts(3 - gy[j], ny, py);
#pragma omp for schedule(static) nowait
            for (int r = 0; r < rows; ++r)
                diff_x_row(gx[j], nx, px, dx, u[j] + (size_t)r * cols, DX[j] + (size_t)r * ndx);
#pragma omp for schedule(static)
            for (int a = 0; a < ndy; ++a)
                diff_y_row(gy[j], ny, py, dy, cols, u[j], a, DY[j] + (size_t)a * cols);
        }
        for (int k = 0; k < nmom; ++k) {
            int even_k = gx[k] == gy[k];
            if ((parity == 0) != even_k) continue;
            const int cols = npts(gx[k], nx, px), rows = npts(gy[k], ny, py);
#pragma omp for schedule(static) nowait
            for (int r = 0; r < rows; ++r) {
                double* w = W[k] + (size_t)r * cols;
                for (int i = 0; i < cols; ++i) w[i] = 0.0;
                for (int j = 0; j < nmom; ++j) {
                    const double mx = Mx[(size_t)k * nmom + j];
                    const double my = My[(size_t)k * nmom + j];
                    if (mx != 0.0) {
                        const double* d = DX[j] + (size_t)r * cols;
                        for (int i = 0; i < cols; ++i) w[i] -= mx * d[i];
                    }
                    if (my != 0.0) {
                        const double* d = DY[j] + (size_t)r * cols;
                        for (int i = 0; i < cols; ++i) w[i] -= my * d[i];
                    }
                }
            }
        }
    }
    for (int j = 0; j < nmom; ++j) { free(DX[j]); free(DY[j]); }
    free(DX);
    free(DY);
    return 0;
}

/*
 * u_k <- u_k + tau * (W_k + q_k - c_k u_k) * E(-c_k tau) for every component k
 * of the given parity (eq. sub_step_solution with r = q + W).  q[k] may be NULL
 * (no source on that component).
 */
int starmap_oracle_update(int nx, int ny, int px, int py, int nmom, const int* gx, const int* gy,
                          int parity, double* const* u, double* const* W,
                          double* const* c, double* const* q, double tau, int emode) {
#pragma omp parallel
    for (int k = 0; k < nmom; ++k) {
        int even_k = gx[k] == gy[k];
        if ((parity == 0) != even_k) continue;
        size_t sz = plane_size(gx, gy, k, nx, ny, px, py);
        double* uk = u[k];
        const double* wk = W[k];
        const double* ck = c[k];
        const double* qk = q ? q[k] : NULL;
#pragma omp for schedule(static) nowait
        for (long long t = 0; t < (long long)sz; ++t) {
            double r = wk[t] + (qk ? qk[t] : 0.0);
            double cc = ck[t];
            uk[t] = uk[t] + tau * (r - cc * uk[t]) * expm1div(-cc * tau, emode);
        }
    }
    return 0;
}
