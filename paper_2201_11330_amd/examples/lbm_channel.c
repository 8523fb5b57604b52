/*
 * A C99 program that drives liblbm.so through include/lbm.h alone: device
 * memory from hipMalloc, the null stream, no Python.  It runs a forced
 * D3Q19 channel (x, z periodic; solid planes y = 0 and ny - 1; halfway
 * bounce-back, Eq. (bb)) from rest at rho = 1, prints the Monitor
 * reductions and the wall force, and writes the final populations f^n
 * ([Q][nz][ny][nx] FP64, little-endian) to the file named on the command
 * line.
 *
 *   lbm_channel OUT.bin [nx ny nz steps]
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "lbm.h"

#define CHECK_LBM(call)                                                                        \
    do {                                                                                       \
        lbm_status st_ = (call);                                                               \
        if (st_ != LBM_OK) {                                                                   \
            fprintf(stderr, "%s: %s (%s)\n", #call, lbm_status_string(st_), lbm_last_error()); \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)

#define CHECK_HIP(call)                                                    \
    do {                                                                   \
        hipError_t e_ = (call);                                            \
        if (e_ != hipSuccess) {                                            \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));     \
            return 1;                                                      \
        }                                                                  \
    } while (0)

int main(int argc, char** argv)
{
    if (argc < 2) {
        fprintf(stderr, "usage: %s OUT.bin [nx ny nz steps]\n", argv[0]);
        return 2;
    }
    const int nx = argc > 2 ? atoi(argv[2]) : 24;
    const int ny = argc > 3 ? atoi(argv[3]) : 18;
    const int nz = argc > 4 ? atoi(argv[4]) : 10;
    const int steps = argc > 5 ? atoi(argv[5]) : 200;
    const size_t N = (size_t)nx * ny * nz;
    const int Q = 19;
    const double force[3] = {1e-5, 0.0, 0.0};
    const lbm_bc bc = {{LBM_PERIODIC, LBM_SOLID_ENDS, LBM_PERIODIC}};

    lbm_ctx* ctx = NULL;
    CHECK_LBM(lbm_create(&ctx, LBM_D3Q19, nx, ny, nz, 0.9, force, &bc, LBM_F64, 0));
    const size_t bytes = lbm_buffer_bytes(ctx);
    void *a = NULL, *b = NULL;
    CHECK_HIP(hipMalloc(&a, bytes));
    CHECK_HIP(hipMalloc(&b, bytes));
    CHECK_LBM(lbm_bind(ctx, a, b, NULL));

    double* h_rho = malloc(sizeof(double) * N);
    double* h_u = calloc(3 * N, sizeof(double));
    double* h_f = malloc(sizeof(double) * Q * N);
    if (!h_rho || !h_u || !h_f) return 1;
    for (size_t i = 0; i < N; ++i) h_rho[i] = 1.0;
    double *d_rho, *d_u, *d_f;
    CHECK_HIP(hipMalloc((void**)&d_rho, sizeof(double) * N));
    CHECK_HIP(hipMalloc((void**)&d_u, sizeof(double) * 3 * N));
    CHECK_HIP(hipMalloc((void**)&d_f, sizeof(double) * Q * N));
    CHECK_HIP(hipMemcpy(d_rho, h_rho, sizeof(double) * N, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_u, h_u, sizeof(double) * 3 * N, hipMemcpyHostToDevice));

    CHECK_LBM(lbm_init_equilibrium(ctx, d_rho, d_u, NULL));
    CHECK_LBM(lbm_step(ctx, steps));
    double mass, ke, umax, wall[3];
    CHECK_LBM(lbm_reduce(ctx, &mass, &ke, &umax));
    CHECK_LBM(lbm_wall_force(ctx, wall));
    CHECK_LBM(lbm_get_populations(ctx, d_f));
    CHECK_HIP(hipMemcpy(h_f, d_f, sizeof(double) * Q * N, hipMemcpyDeviceToHost));
    printf("steps %lld mass %.17g ke %.17g umax %.17g wall_force %.17g %.17g %.17g\n",
           lbm_steps_taken(ctx), mass, ke, umax, wall[0], wall[1], wall[2]);

    FILE* fh = fopen(argv[1], "wb");
    if (!fh || fwrite(h_f, sizeof(double), (size_t)Q * N, fh) != (size_t)Q * N) {
        fprintf(stderr, "cannot write %s\n", argv[1]);
        return 1;
    }
    fclose(fh);

    CHECK_LBM(lbm_destroy(ctx));
    CHECK_HIP(hipFree(a));
    CHECK_HIP(hipFree(b));
    CHECK_HIP(hipFree(d_rho));
    CHECK_HIP(hipFree(d_u));
    CHECK_HIP(hipFree(d_f));
    free(h_rho);
    free(h_u);
    free(h_f);
    return 0;
}
