/* Exercises every entry point of the oracle (oracle/yyo.h) on small and
 * ragged grids, for a build with AddressSanitizer and UndefinedBehavior-
 * Sanitizer (tests/test_oracle_sanitized.py compiles and runs it on the
 * CPU).  Exit status 0 and no sanitizer report mean every access stayed in
 * bounds and no undefined operation occurred. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "yyo.h"

static unsigned long long lcg = 12345;
static double rnd(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) / 9007199254740992.0 * 2.0 - 1.0;
}

static void fill_rand(double *a, int64_t n, double s)
{
    for (int64_t q = 0; q < n; q++) a[q] = s * rnd();
}

static int run(int nr, int nt, int np, double delta, int mode, int extras)
{
    yyo *h = yyo_create(nr, nt, np, 0.5, 1.0, delta);
    if (!h) return 1;
    if (yyo_set_params(h, 1.0, 1e3, 2e-3, 1.0, 1.0, 0.0)) return 2;
    yyo_set_mode(h, mode);
    const int64_t npad = yyo_field_count(h, YYO_T, YYO_PADDED);
    double *buf = malloc(sizeof(double) * npad), *out = malloc(sizeof(double) * npad);
    for (int f = 0; f < YYO_NF; f++)
        for (int l = 0; l < 3; l++) {
            const int64_t n = yyo_field_count(h, f, YYO_MAC);
            fill_rand(buf, n, 0.01);
            yyo_set_field(h, f, l, YYO_MAC, buf);
        }
    for (int f = YYO_T; f <= YYO_U1P; f++) {
        const int64_t n = yyo_field_count(h, f, YYO_MAC);
        fill_rand(buf, n, 0.1);
        yyo_set_forcing(h, f, buf);
    }
    if (extras) {
        yyo_set_mass_fix(h, 1);
        yyo_set_mass_fix_params(h, 1e-3, 0.0);
        yyo_set_pressure_exchange(h, 1);
        yyo_set_t_bc(h, 1, 1.0, 0.5);
        const int64_t nw = 2 * (int64_t)(nt + 2) * (np + 2);
        double *w = malloc(sizeof(double) * nw);
        for (int c = YYO_T; c <= YYO_U1P; c++)
            for (int l = 0; l < 3; l++)
                for (int side = 0; side < 2; side++) {
                    fill_rand(w, nw, 0.01);
                    yyo_set_wall(h, c, l, side, w);
                }
        free(w);
    }
    yyo_fill(h, YYO_LEV_N);
    yyo_extrapolate(h);
    fill_rand(buf, npad, 1.0);
    for (int f = 0; f < YYO_NF; f++) {
        if (f == YYO_P1 || f == YYO_P2) continue;
        for (int d = 0; d < 3; d++) yyo_sweep(h, f, d, buf, out);
        for (int op = YYO_OP_DRR; op <= YYO_OP_LP; op++) yyo_apply_op(h, f, op, buf, out);
        yyo_residual(h, f, out);
    }
    for (int op = YYO_OP_DRR; op <= YYO_OP_DPP_HAT; op++) yyo_sweep_op(h, op, buf, out);
    yyo_step(h, 2);
    if (extras) {
        const int64_t nw = 2 * (int64_t)(nt + 2) * (np + 2);
        double *w = malloc(sizeof(double) * nw);
        for (int c = YYO_T; c <= YYO_U1P; c++)
            for (int side = 0; side < 2; side++) {
                fill_rand(w, nw, 0.01);
                yyo_set_wall(h, c, YYO_LEV_K, side, w);
            }
        free(w);
    }
    int k = yyo_step_tol(h, 5, 1e-30);
    double norms[5 * 2 * 10];
    yyo_get_norms(h, norms, 5 * 2 * 10);
    for (int f = 0; f < YYO_NF; f++) {
        yyo_get_field(h, f, YYO_LEV_N, YYO_MAC, out);
        yyo_get_field(h, f, YYO_LEV_N, YYO_PADDED, out);
    }
    free(buf);
    free(out);
    yyo_destroy(h);
    return k == 5 ? 0 : 3;
}

int main(void)
{
    double lo[8], di[8], up[8], rhs[8], x[8];
    for (int i = 0; i < 8; i++) { lo[i] = rnd(); up[i] = rnd(); di[i] = 4.0 + rnd(); rhs[i] = rnd(); }
    yyo_thomas(8, lo, di, up, rhs, x);
    int rc = 0;
    rc |= run(4, 12, 36, 0.0, 0, 0);
    rc |= run(3, 13, 37, 0.0, 1, 1);
    rc |= run(5, 16, 40, 0.15, 0, 1);
    printf("sanitized oracle run: %s\n", rc ? "FAILED" : "ok");
    return rc;
}
