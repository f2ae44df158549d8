/* A plain C caller of the library: everything through include/psm.h and the
 * HIP runtime, no Python or torch. Reads a box and its spheres from a text
 * file, runs a number of steps from rest (rho = 1, u = 0) and prints the
 * per-sphere force and torque, the FP64 mass and the density and velocity of
 * cell 0. Input file: nx ny nz tau fx fy fz steps n, then n lines of
 * x y z r Ux Uy Uz Ox Oy Oz. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "psm.h"

#define HIPCHECK(call)                                                           \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            fprintf(stderr, "HIP error %d at line %d\n", (int)e_, __LINE__);     \
            return 2;                                                            \
        }                                                                        \
    } while (0)
#define PSMCHECK(call)                                                           \
    do {                                                                         \
        int s_ = (call);                                                         \
        if (s_ != PSM_OK) {                                                      \
            fprintf(stderr, "psm error %d: %s\n", s_, psm_last_error());         \
            return 3;                                                            \
        }                                                                        \
    } while (0)

int main(int argc, char** argv) {
    psm_box_desc d;
    int steps = 0, n = 0, i;
    FILE* fh;
    double *x, *r, *U, *O, *F, *T, *u_dev = NULL, *rho_dev = NULL, rho0 = 0.0, u0[3];
    void* ws = NULL;
    size_t bytes = 0;
    psm_ctx* ctx = NULL;
    double mass = 0.0;
    long long overflows = 0;
    long long N;

    if (argc != 2 || !(fh = fopen(argv[1], "r"))) return 1;
    memset(&d, 0, sizeof d);
    if (fscanf(fh, "%d %d %d %lf %lf %lf %lf %d %d", &d.nx, &d.ny, &d.nz, &d.tau, &d.fext[0], &d.fext[1],
               &d.fext[2], &steps, &n) != 9)
        return 1;
    x = malloc(sizeof(double) * 3 * (n + 1));
    r = malloc(sizeof(double) * (n + 1));
    U = malloc(sizeof(double) * 3 * (n + 1));
    O = malloc(sizeof(double) * 3 * (n + 1));
    F = malloc(sizeof(double) * 3 * (n + 1));
    T = malloc(sizeof(double) * 3 * (n + 1));
    d.max_radius = 0.0;
    for (i = 0; i < n; ++i) {
        if (fscanf(fh, "%lf %lf %lf %lf %lf %lf %lf %lf %lf %lf", &x[3 * i], &x[3 * i + 1], &x[3 * i + 2], &r[i],
                   &U[3 * i], &U[3 * i + 1], &U[3 * i + 2], &O[3 * i], &O[3 * i + 1], &O[3 * i + 2]) != 10)
            return 1;
        if (r[i] > d.max_radius) d.max_radius = r[i];
    }
    fclose(fh);
    d.max_particles = n;
    d.mapping = PSM_MAP_LINEAR;
    d.subsample_n = 4;
    N = (long long)d.nx * d.ny * d.nz;

    PSMCHECK(psm_workspace_size(&d, 1, PSM_FP64, &bytes));
    HIPCHECK(hipMalloc(&ws, bytes));
    HIPCHECK(hipMalloc((void**)&u_dev, sizeof(double) * 3 * N));
    HIPCHECK(hipMalloc((void**)&rho_dev, sizeof(double) * N));
    HIPCHECK(hipMemset(u_dev, 0, sizeof(double) * 3 * N));
    PSMCHECK(psm_create(&d, 1, PSM_FP64, 0.0, NULL, ws, bytes, &ctx));
    PSMCHECK(psm_set_equilibrium(ctx, 0, NULL, u_dev));
    PSMCHECK(psm_set_particles(ctx, 0, n, x, r, U, O));
    PSMCHECK(psm_step(ctx, steps));
    PSMCHECK(psm_get_forces(ctx, 0, F, T));
    PSMCHECK(psm_get_stats(ctx, 0, &mass, NULL, &overflows));
    PSMCHECK(psm_get_macroscopic(ctx, 0, rho_dev, u_dev));
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(&rho0, rho_dev, sizeof(double), hipMemcpyDeviceToHost));
    for (i = 0; i < 3; ++i) HIPCHECK(hipMemcpy(&u0[i], u_dev + i * N, sizeof(double), hipMemcpyDeviceToHost));
    /* an argument error is reported, not thrown */
    if (psm_step(ctx, -1) != PSM_EINVAL) return 4;
    PSMCHECK(psm_destroy(ctx));
    HIPCHECK(hipFree(ws));
    HIPCHECK(hipFree(u_dev));
    HIPCHECK(hipFree(rho_dev));
    for (i = 0; i < n; ++i)
        printf("sphere %d %.17g %.17g %.17g %.17g %.17g %.17g\n", i, F[3 * i], F[3 * i + 1], F[3 * i + 2],
               T[3 * i], T[3 * i + 1], T[3 * i + 2]);
    printf("mass %.17g\n", mass);
    printf("cell0 %.17g %.17g %.17g %.17g\n", rho0, u0[0], u0[1], u0[2]);
    printf("overflows %lld\n", overflows);
    free(x); free(r); free(U); free(O); free(F); free(T);
    return 0;
}
