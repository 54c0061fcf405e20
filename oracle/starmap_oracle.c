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
 * Plain loops; OpenMP only splits independent rows, so results are identical
 * for any thread count.
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
   mode 1: the paper's switch (Sect. 5.5): a three-term Taylor series below
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
 * D_x of a field on grid (tx, ty) -> field on grid (3 - tx, ty).
 * The source row is first extended by the boundary rule, then differenced:
 *   tx == 1 (cells 1..n, result on nodes p..n): extended cells p..n+1 with
 *           ghost cell 0 := cell 1 (extrapolation) and ghost cell n+1 := cell n
 *           (extrapolation) or := cell 1 (periodic);
 *   tx == 2 (nodes p..n, result on cells 1..n): extended nodes 0..n with
 *           node 0 := node n (periodic); extrapolation has node 0 already.
 * Result(a) = (ext(a+1) - ext(a)) / h for a = 0 .. (result points - 1).
 */
static void diff_x(int tx, int ty, int nx, int ny, int px, int py, double dx,
                   const double* src, double* dst) {
    const int ns = npts(tx, nx, px);
    const int nd = npts(3 - tx, nx, px);
    const int rows = npts(ty, ny, py);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < rows; ++j) {
        const double* s = src + (size_t)j * ns;
        double* d = dst + (size_t)j * nd;
        double* ext = (double*)malloc(sizeof(double) * (size_t)(nd + 1));
        for (int a = 0; a <= nd; ++a) {
            double v;
            if (tx == 1) {
                int ci = px + a;                     /* paper cell index, 0..n+1 */
                if (ci == 0) v = s[0];               /* ghost left (extrapolation) */
                else if (ci == nx + 1) v = px ? s[0] : s[nx - 1];
                else v = s[ci - 1];
            } else {
                int ni = a;                          /* paper node index 0..n */
                if (ni == 0 && px) v = s[nx - 1];    /* node 0 := node n (periodic) */
                else v = s[ni - px];
            }
            ext[a] = v;
        }
        for (int a = 0; a < nd; ++a) d[a] = (ext[a + 1] - ext[a]) / dx;
        free(ext);
    }
}

/* D_y: the same rule along y; field on grid (tx, ty) -> grid (tx, 3 - ty). */
static void diff_y(int tx, int ty, int nx, int ny, int px, int py, double dy,
                   const double* src, double* dst) {
    const int cols = npts(tx, nx, px);
    const int nd = npts(3 - ty, ny, py);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < cols; ++i) {
        double* ext = (double*)malloc(sizeof(double) * (size_t)(nd + 1));
        for (int a = 0; a <= nd; ++a) {
            double v;
            if (ty == 1) {
                int ci = py + a;
                if (ci == 0) v = src[i];
                else if (ci == ny + 1) v = py ? src[i] : src[(size_t)(ny - 1) * cols + i];
                else v = src[(size_t)(ci - 1) * cols + i];
            } else {
                int ni = a;
                if (ni == 0 && py) v = src[(size_t)(ny - 1) * cols + i];
                else v = src[(size_t)(ni - py) * cols + i];
            }
            ext[a] = v;
        }
        for (int a = 0; a < nd; ++a) dst[(size_t)a * cols + i] = (ext[a + 1] - ext[a]) / dy;
        free(ext);
    }
}

static size_t plane_size(const int* gx, const int* gy, int k, int nx, int ny, int px, int py) {
    return (size_t)npts(gx[k], nx, px) * (size_t)npts(gy[k], ny, py);
}

/*
 * W_k = - sum_j Mx(k,j) D_x u_j - sum_j My(k,j) D_y u_j for every component k
 * of the given parity (even: G11 and G22; odd: G21 and G12).  Only the nonzero
 * entries of the rows are visited.  W[k] must hold k's grid size for those k.
 * Returns 0, or -1 if a nonzero entry couples grids that the staggering does
 * not allow.
 */
int starmap_oracle_flux(int nx, int ny, int px, int py, double dx, double dy, int nmom,
                        const int* gx, const int* gy, const double* Mx, const double* My,
                        int parity, double* const* u, double* const* W) {
    /* differences of all components of the other parity, computed once each */
    double** DX = (double**)calloc((size_t)nmom, sizeof(double*));
    double** DY = (double**)calloc((size_t)nmom, sizeof(double*));
    int status = 0;
    for (int j = 0; j < nmom; ++j) {
        int even_j = gx[j] == gy[j];
        if ((parity == 0) == even_j) continue;  /* same parity as the outputs */
        size_t szx = (size_t)npts(3 - gx[j], nx, px) * (size_t)npts(gy[j], ny, py);
        size_t szy = (size_t)npts(gx[j], nx, px) * (size_t)npts(3 - gy[j], ny, py);
        DX[j] = (double*)malloc(sizeof(double) * szx);
        DY[j] = (double*)malloc(sizeof(double) * szy);
        diff_x(gx[j], gy[j], nx, ny, px, py, dx, u[j], DX[j]);
        diff_y(gx[j], gy[j], nx, ny, px, py, dy, u[j], DY[j]);
    }
    for (int k = 0; k < nmom && status == 0; ++k) {
        int even_k = gx[k] == gy[k];
        if ((parity == 0) != even_k) continue;
        size_t sz = plane_size(gx, gy, k, nx, ny, px, py);
        double* w = W[k];
        for (size_t t = 0; t < sz; ++t) w[t] = 0.0;
        for (int j = 0; j < nmom; ++j) {
            double mx = Mx[(size_t)k * nmom + j];
            double my = My[(size_t)k * nmom + j];
            if (mx != 0.0) {
                if (!DX[j] || 3 - gx[j] != gx[k] || gy[j] != gy[k]) { status = -1; break; }
                const double* d = DX[j];
#pragma omp parallel for schedule(static)
                for (long long t = 0; t < (long long)sz; ++t) w[t] -= mx * d[t];
            }
            if (my != 0.0) {
                if (!DY[j] || gx[j] != gx[k] || 3 - gy[j] != gy[k]) { status = -1; break; }
                const double* d = DY[j];
#pragma omp parallel for schedule(static)
                for (long long t = 0; t < (long long)sz; ++t) w[t] -= my * d[t];
            }
        }
    }
    for (int j = 0; j < nmom; ++j) { free(DX[j]); free(DY[j]); }
    free(DX);
    free(DY);
    return status;
}

/*
 * u_k <- u_k + tau * (W_k + q_k - c_k u_k) * E(-c_k tau) for every component k
 * of the given parity (eq. sub_step_solution with r = q + W).  q[k] may be NULL
 * (no source on that component).
 */
int starmap_oracle_update(int nx, int ny, int px, int py, int nmom, const int* gx, const int* gy,
                          int parity, double* const* u, double* const* W,
                          double* const* c, double* const* q, double tau, int emode) {
    for (int k = 0; k < nmom; ++k) {
        int even_k = gx[k] == gy[k];
        if ((parity == 0) != even_k) continue;
        size_t sz = plane_size(gx, gy, k, nx, ny, px, py);
        double* uk = u[k];
        const double* wk = W[k];
        const double* ck = c[k];
        const double* qk = q ? q[k] : NULL;
#pragma omp parallel for schedule(static)
        for (long long t = 0; t < (long long)sz; ++t) {
            double r = wk[t] + (qk ? qk[t] : 0.0);
            double cc = ck[t];
            uk[t] = uk[t] + tau * (r - cc * uk[t]) * expm1div(-cc * tau, emode);
        }
    }
    return 0;
}
