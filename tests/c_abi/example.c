/*
 * The C ABI used from plain C (no Python): a planar fault of N elements,
 * device buffers from hipMalloc -- the slip rates and tractions, the scratch
 * of the FDP=H window scan and each operator's workspace (the library
 * allocates no device memory) -- results copied back and printed one value
 * per line.
 *
 *   example N M            the plain form and the FDP=H form on the same
 *                          input: the plain form's M x N tractions, then the
 *                          FDP=H form's
 *   example N M scenarios  one FDP=H operator carrying two slip-rate
 *                          histories (n_rhs = 2): M x 2N tractions, rows
 *                          holding scenario 0's N values, then scenario 1's
 *   example N M rupture    dynamic rupture on the plain form (exponential
 *                          slip weakening, t_th = 1e-2, t_dy = 0, d_c = 0.05;
 *                          initial traction 0.35e-2, 1.01e-2 on the 20
 *                          central elements): the M x N slip rates
 *
 * Slip rate: D[n][j] = sin(0.37 j + 0.11 n) + 0.5 cos(0.05 j n), the second
 * scenario cos(0.21 j - 0.07 n) (no random numbers, so the reader can
 * regenerate them).
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

static void fdph_defaults(bie_fdph_params *q) {
    q->eta = 2.0;
    q->leaf_size = 32;
    q->n_c = 20;
    q->eps_aca = 1e-8;
    q->eps_q = 1e-3;
    q->eps_st = 1e-6;
    q->precision = BIE_FP64;
    q->seed = 7;
}

/* Plain form: plan, workspace of the reported size, operator inside it. */
static int build_dense(const bie_problem *p, bie_op **op, void **ws) {
    bie_plan *plan = NULL;
    int64_t bytes = 0;
    CHECK(bie_plan_dense(p, &plan));
    CHECK(bie_workspace_size(plan, &bytes));
    if (hipMalloc(ws, (size_t)bytes) != hipSuccess) return 3;
    CHECK(bie_build_kernel(plan, *ws, bytes, NULL, op));
    bie_plan_free(plan);
    return 0;
}

/* FDP=H form: plan (host), window scan in a scratch buffer, workspace. */
static int build_fdph(const bie_problem *p, const bie_fdph_params *q, bie_op **op, void **ws) {
    bie_plan *plan = NULL;
    int64_t sbytes = 0, bytes = 0;
    void *scratch = NULL;
    CHECK(bie_plan_fdph(p, 1, q, &plan));
    CHECK(bie_plan_scratch_size(plan, &sbytes));
    if (sbytes > 0 && hipMalloc(&scratch, (size_t)sbytes) != hipSuccess) return 3;
    CHECK(bie_plan_windows(plan, scratch, sbytes, NULL));
    if (scratch) (void)hipFree(scratch);
    CHECK(bie_workspace_size(plan, &bytes));
    if (hipMalloc(ws, (size_t)bytes) != hipSuccess) return 3;
    CHECK(bie_compress_fdph(plan, *ws, bytes, NULL, op));
    bie_plan_free(plan);
    return 0;
}

/* Two slip-rate histories through one FDP=H operator (n_rhs = 2). */
static int run_scenarios(const bie_problem *p, const double *D, int N, int M) {
    const size_t R = 2, row = R * (size_t)N;
    double *D2 = malloc(sizeof(double) * (size_t)M * row), *T2 = malloc(sizeof(double) * (size_t)M * row);
    for (int n = 0; n < M; ++n)
        for (int j = 0; j < N; ++j) {
            D2[(size_t)n * row + j] = D[(size_t)n * N + j];
            D2[(size_t)n * row + N + j] = cos(0.21 * j - 0.07 * n);
        }
    double *dD = NULL, *dT = NULL;
    if (hipMalloc((void **)&dD, sizeof(double) * (size_t)M * row) != hipSuccess) return 3;
    if (hipMalloc((void **)&dT, sizeof(double) * (size_t)M * row) != hipSuccess) return 3;
    if (hipMemcpy(dD, D2, sizeof(double) * (size_t)M * row, hipMemcpyHostToDevice) != hipSuccess) return 3;
    bie_fdph_params q = {0};
    fdph_defaults(&q);
    q.n_rhs = 2;
    bie_op *op = NULL;
    void *ws = NULL;
    if (build_fdph(p, &q, &op, &ws)) return 1;
    CHECK(bie_run(op, dD, dT, M, NULL));
    if (hipMemcpy(T2, dT, sizeof(double) * (size_t)M * row, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    for (size_t k = 0; k < (size_t)M * row; ++k) printf("%.17g\n", T2[k]);
    bie_destroy(op);
    (void)hipFree(ws);
    (void)hipFree(dD);
    (void)hipFree(dT);
    free(D2);
    free(T2);
    return 0;
}

/* Dynamic rupture on the plain form: coupled steps with exponential slip
 * weakening. */
static int run_rupture(const bie_problem *p, int N, int M) {
    double *t0 = malloc(sizeof(double) * N), *Dh = malloc(sizeof(double) * (size_t)M * N);
    for (int j = 0; j < N; ++j) t0[j] = (j >= N / 2 - 10 && j < N / 2 + 10) ? 1.01e-2 : 0.35e-2;
    double *dt0 = NULL, *dslip = NULL, *dD = NULL, *dT = NULL;
    int32_t *dstate = NULL;
    if (hipMalloc((void **)&dt0, sizeof(double) * N) != hipSuccess) return 3;
    if (hipMalloc((void **)&dslip, sizeof(double) * N) != hipSuccess) return 3;
    if (hipMalloc((void **)&dstate, sizeof(int32_t) * N) != hipSuccess) return 3;
    if (hipMalloc((void **)&dD, sizeof(double) * (size_t)M * N) != hipSuccess) return 3;
    if (hipMalloc((void **)&dT, sizeof(double) * (size_t)M * N) != hipSuccess) return 3;
    if (hipMemcpy(dt0, t0, sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess) return 3;
    if (hipMemset(dslip, 0, sizeof(double) * N) != hipSuccess) return 3;
    if (hipMemset(dstate, 0, sizeof(int32_t) * N) != hipSuccess) return 3;
    bie_op *op = NULL;
    void *ws = NULL;
    if (build_dense(p, &op, &ws)) return 1;
    bie_friction fr = {0};
    fr.law = BIE_LAW_EXP_WEAKENING;
    fr.t_th = 1e-2;
    fr.t_dy = 0.0;
    fr.d_c = 0.05;
    CHECK(bie_rupture_run(op, &fr, dt0, dslip, dstate, dD, dT, M, NULL));
    if (hipMemcpy(Dh, dD, sizeof(double) * (size_t)M * N, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    for (size_t k = 0; k < (size_t)M * N; ++k) printf("%.17g\n", Dh[k]);
    bie_destroy(op);
    (void)hipFree(ws);
    (void)hipFree(dt0);
    (void)hipFree(dslip);
    (void)hipFree(dstate);
    (void)hipFree(dD);
    (void)hipFree(dT);
    free(t0);
    free(Dh);
    return 0;
}

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

    const char *mode = argc > 3 ? argv[3] : "plain";
    if (mode[0] == 's') return run_scenarios(&p, D, N, M);
    if (mode[0] == 'r') return run_rupture(&p, N, M);

    bie_op *dense = NULL, *fdph = NULL;
    void *ws_dense = NULL, *ws_fdph = NULL;
    if (build_dense(&p, &dense, &ws_dense)) return 1;
    CHECK(bie_run(dense, dD, dT, M, NULL));
    if (hipMemcpy(T, dT, sizeof(double) * (size_t)M * N, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    for (size_t k = 0; k < (size_t)M * N; ++k) printf("%.17g\n", T[k]);

    bie_fdph_params q = {0};
    fdph_defaults(&q);
    if (build_fdph(&p, &q, &fdph, &ws_fdph)) return 1;
    CHECK(bie_reset(fdph, NULL));
    CHECK(bie_run(fdph, dD, dT, M, NULL));
    if (hipMemcpy(T, dT, sizeof(double) * (size_t)M * N, hipMemcpyDeviceToHost) != hipSuccess) return 3;
    for (size_t k = 0; k < (size_t)M * N; ++k) printf("%.17g\n", T[k]);
    bie_stats st;
    CHECK(bie_query(fdph, &st));
    fprintf(stderr, "fdph: %lld admissible leaves, %lld near pairs\n", (long long)st.n_adm, (long long)st.near_pairs);

    bie_destroy(dense);
    bie_destroy(fdph);
    (void)hipFree(ws_dense);
    (void)hipFree(ws_fdph);
    (void)hipFree(dD);
    (void)hipFree(dT);
    free(xa);
    free(xb);
    free(D);
    free(T);
    return 0;
}
