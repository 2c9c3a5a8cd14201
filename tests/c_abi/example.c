/*
 * The C ABI used from plain C (no Python): a planar fault of N elements,
 * the plain form and the FDP=H form on the same input, device buffers from
 * hipMalloc, tractions copied back and printed (one value per line, the
 * plain form's M x N values, then the FDP=H form's).
 *
 * Slip rate: D[n][j] = sin(0.37 j + 0.11 n) + 0.5 cos(0.05 j n) (no random
 * numbers, so the reader can regenerate it).
 *
 * Usage: example N M
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "bie.h"

#define CHECK(x)                                                          \
    do {                                                                  \
        int rc_ = (x);                                                    \
        if (rc_ != BIE_OK) {                                              \
            fprintf(stderr, "%s failed (%d): %s\n", #x, rc_, bie_last_error()); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(int argc, char **argv) {
    if (argc < 3) return 2;
    const int N = atoi(argv[1]), M = atoi(argv[2]);
    double *xa = malloc(sizeof(double) * 2 * N), *xb = malloc(sizeof(double) * 2 * N);
    double *D = malloc(sizeof(double) * (size_t)M * N), *T = malloc(sizeof(double) * (size_t)M * N);
    for (int j = 0; j < N; ++j) {
        xa[2 * j] = j;
        xa[2 * j + 1] = 0.0;
        xb[2 * j] = j + 1;
        xb[2 * j + 1] = 0.0;
    }
    for (int n = 0; n < M; ++n)
        for (int j = 0; j < N; ++j) D[(size_t)n * N + j] = sin(0.37 * j + 0.11 * n) + 0.5 * cos(0.05 * j * n);
    bie_problem p = {0};
    p.n_elem = N;
    p.n_lags = M;
    p.xa_host = xa;
    p.xb_host = xb;
    p.mu = 1.0;
    p.beta = 1.0;
    p.dt = 0.5;
    p.eps_t = 1.0;
    p.mode = BIE_MODE_ANTIPLANE;

    double *dD = NULL, *dT = NULL;
    if (hipMalloc((void **)&dD, sizeof(double) * (size_t)M * N) != hipSuccess) return 3;
    if (hipMalloc((void **)&dT, sizeof(double) * (size_t)M * N) != hipSuccess) return 3;
    if (hipMemcpy(dD, D, sizeof(double) * (size_t)M * N, hipMemcpyHostToDevice) != hipSuccess) return 3;

    bie_op *dense = NULL, *fdph = NULL;
    CHECK(bie_build_kernel(&p, NULL, &dense));
    CHECK(bie_run(dense, dD, dT, M, NULL));
    if (hipMemcpy(T, dT, sizeof(double) * (size_t)M * N, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    for (size_t k = 0; k < (size_t)M * N; ++k) printf("%.17g\n", T[k]);

    bie_fdph_params q = {0};
    q.eta = 2.0;
    q.leaf_size = 32;
    q.n_c = 20;
    q.eps_aca = 1e-8;
    q.eps_q = 1e-3;
    q.eps_st = 1e-6;
    q.precision = BIE_FP64;
    q.seed = 7;
    CHECK(bie_compress_fdph(&p, &q, NULL, &fdph));
    CHECK(bie_reset(fdph, NULL));
    CHECK(bie_run(fdph, dD, dT, M, NULL));
    if (hipMemcpy(T, dT, sizeof(double) * (size_t)M * N, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    for (size_t k = 0; k < (size_t)M * N; ++k) printf("%.17g\n", T[k]);
    bie_stats st;
    CHECK(bie_query(fdph, &st));
    fprintf(stderr, "fdph: %lld admissible leaves, %lld near pairs\n", (long long)st.n_adm, (long long)st.near_pairs);

    bie_destroy(dense);
    bie_destroy(fdph);
    (void)hipFree(dD);
    (void)hipFree(dT);
    free(xa);
    free(xb);
    free(D);
    free(T);
    return 0;
}
