/* Runs every oracle entry point once on small 2D and 3D grids (both time
 * orders, both tap kinds, a medium with both attenuation laws, the PML), for
 * the address and undefined-behaviour sanitizer build of the oracle in
 * tests/test_sanitizers.py.  Prints "ok" and exits 0 when every call
 * returns 0; a sanitizer report aborts the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/stride_oracle.h"

static int fails = 0;

static void check(int rc, const char *what)
{
    if (rc != 0) {
        printf("%s returned %d\n", what, rc);
        fails++;
    }
}

static void run(int ndim, int order, int torder, int interp)
{
    oracle_grid_t g = {0};
    g.ndim = ndim;
    long n[3] = {14, 17, 12};
    for (int a = 0; a < 3; a++) {
        g.shape[a] = a < ndim ? n[a] : 1;
        g.spacing[a] = 0.5e-3;
    }
    g.space_order = order;
    g.nb = 5;
    g.vref = 1500.0;
    g.dt = 0.25 * 0.5e-3 / 1600.0;
    g.nt = 23;
    g.time_order = torder;
    g.interp = interp;
    long np3[3];
    long N = oracle_padded_points(&g, np3);
    long nphys = g.shape[0] * g.shape[1] * g.shape[2];
    double *vp = malloc(sizeof(double) * nphys), *rho = malloc(sizeof(double) * nphys);
    double *al = malloc(sizeof(double) * nphys), *dvp = malloc(sizeof(double) * nphys);
    double *pad = malloc(sizeof(double) * N), *lu = malloc(sizeof(double) * N);
    for (long i = 0; i < nphys; i++) {
        vp[i] = 1500.0 + 100.0 * sin(0.37 * i);
        rho[i] = 1000.0 + 200.0 * cos(0.21 * i);
        al[i] = 5.0 + 4.0 * sin(0.11 * i);
    }
    double src[3] = {6.3e-3, 4.1e-3, 3.3e-3}, rec[6] = {2.2e-3, 5.5e-3, 4.0e-3, 4.4e-3, 1.3e-3, 2.0e-3};
    int nt = g.nt;
    double *wav = calloc(nt, sizeof(double)), *tr = calloc(2 * nt, sizeof(double));
    double *obs = calloc(2 * nt, sizeof(double)), *dw = calloc(nt, sizeof(double));
    for (int t = 0; t < nt; t++)
        wav[t] = sin(0.4 * t) * exp(-0.01 * t * t);
    check(oracle_pad(&g, vp, pad) , "pad");
    check(oracle_pad_transpose(&g, pad, dvp), "pad_transpose");
    check(oracle_eta(&g, lu), "eta");
    check(oracle_laplacian(&g, pad, lu), "laplacian");
    int T = oracle_taps_per_point(&g);
    long *idx = malloc(sizeof(long) * T * 2);
    double *w = malloc(sizeof(double) * T * 2);
    check(oracle_taps(&g, 2, rec, idx, w), "taps");
    check(oracle_forward(&g, vp, 1, src, wav, 2, rec, tr, 0, NULL, NULL), "forward");
    check(oracle_adjoint(&g, vp, 1, src, wav, 2, rec, tr, dvp, dw, 4), "adjoint");
    double J = 0.0;
    check(oracle_gradient(&g, vp, 1, src, wav, 2, rec, obs, tr, &J, dvp, 0), "gradient");
    if (torder != 4) {
        for (int y = 0; y <= 2; y += 2) {
            check(oracle_forward_medium(&g, vp, rho, al, y, 1, src, wav, 2, rec, tr), "forward_medium");
            check(oracle_adjoint_medium(&g, vp, rho, al, y, 1, src, wav, 2, rec, tr, dvp, dw, 5),
                  "adjoint_medium");
            check(oracle_gradient_medium(&g, vp, rho, NULL, y, 1, src, wav, 2, rec, obs, tr, &J, dvp, 0),
                  "gradient_medium");
        }
        check(oracle_forward_pml(&g, vp, 1, src, wav, 2, rec, tr), "forward_pml");
    }
    check(oracle_lowpass(tr, obs, 2, nt, g.dt, 4e5) < 0, "lowpass");
    free(vp); free(rho); free(al); free(dvp); free(pad); free(lu); free(idx); free(w);
    free(wav); free(tr); free(obs); free(dw);
}

int main(void)
{
    for (int nd = 2; nd <= 3; nd++)
        for (int order = 8; order <= 10; order += 2)
            for (int torder = 2; torder <= 4; torder += 2)
                for (int interp = 0; interp <= 1; interp++)
                    run(nd, order, torder, interp);
    if (fails)
        return 1;
    printf("ok\n");
    return 0;
}
