/*
 * Runs the oracle's half-step functions under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only; test infrastructure).
 *
 * Reads from stdin: nx ny px py nmom, then gx[nmom], gy[nmom], then the dense
 * Mx and My (nmom x nmom each, row-major), then every component's initial
 * values on its own grid (moment order).  Applies S^o_{tau} S^e_{tau}
 * S^o_{tau} with decay c = 1 + k/10 and a source on component 0, and prints
 * the final values (%.17g, moment order).
 */
#include "../oracle/starmap_oracle.c"

#include <stdio.h>

int main(void) {
    int nx, ny, px, py, nmom;
    if (scanf("%d %d %d %d %d", &nx, &ny, &px, &py, &nmom) != 5) return 2;
    int* gx = (int*)malloc(sizeof(int) * (size_t)nmom);
    int* gy = (int*)malloc(sizeof(int) * (size_t)nmom);
    for (int k = 0; k < nmom; ++k) if (scanf("%d", &gx[k]) != 1) return 2;
    for (int k = 0; k < nmom; ++k) if (scanf("%d", &gy[k]) != 1) return 2;
    double* Mx = (double*)malloc(sizeof(double) * (size_t)nmom * (size_t)nmom);
    double* My = (double*)malloc(sizeof(double) * (size_t)nmom * (size_t)nmom);
    for (int i = 0; i < nmom * nmom; ++i) if (scanf("%lf", &Mx[i]) != 1) return 2;
    for (int i = 0; i < nmom * nmom; ++i) if (scanf("%lf", &My[i]) != 1) return 2;
    double** u = (double**)malloc(sizeof(double*) * (size_t)nmom);
    double** W = (double**)malloc(sizeof(double*) * (size_t)nmom);
    double** c = (double**)malloc(sizeof(double*) * (size_t)nmom);
    double** q = (double**)malloc(sizeof(double*) * (size_t)nmom);
    for (int k = 0; k < nmom; ++k) {
        size_t sz = plane_size(gx, gy, k, nx, ny, px, py);
        u[k] = (double*)malloc(sizeof(double) * sz);
        W[k] = (double*)malloc(sizeof(double) * sz);
        c[k] = (double*)malloc(sizeof(double) * sz);
        q[k] = k == 0 ? (double*)malloc(sizeof(double) * sz) : NULL;
        for (size_t t = 0; t < sz; ++t) {
            if (scanf("%lf", &u[k][t]) != 1) return 2;
            c[k][t] = 1.0 + 0.1 * k;
            if (q[k]) q[k][t] = 0.5;
        }
    }
    const double dx = 1.0 / nx, dy = 1.0 / ny, tau = 0.25 * dx;
    const int order[3] = {1, 0, 1};
    for (int s = 0; s < 3; ++s) {
        if (starmap_oracle_flux(nx, ny, px, py, dx, dy, nmom, gx, gy, Mx, My, order[s], u, W)) return 3;
        starmap_oracle_update(nx, ny, px, py, nmom, gx, gy, order[s], u, W, c, q, tau, s == 2);
    }
    for (int k = 0; k < nmom; ++k) {
        size_t sz = plane_size(gx, gy, k, nx, ny, px, py);
        for (size_t t = 0; t < sz; ++t) printf("%.17g\n", u[k][t]);
        free(u[k]);
        free(W[k]);
        free(c[k]);
        free(q[k]);
    }
    free(u); free(W); free(c); free(q); free(Mx); free(My); free(gx); free(gy);
    return 0;
}
