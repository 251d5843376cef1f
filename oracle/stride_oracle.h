/*
 * stride_oracle.h -- plain FP64 CPU oracle for the acoustic FWI hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source with the HIP path.
 *
 * What it computes (all in double precision, plain loops, OpenMP over the
 * outermost grid axis only):
 *   - the constant-density, lossless acoustic wave equation
 *         (1/vp^2) d2p/dt2 = lap(p) + s                          (Sec. 2.4, acoustic
 *     equation with rho constant and alpha0 = 0)
 *     stepped by second-order leapfrog in time and a 2r-order central Laplacian,
 *     r in 1..5 (Sec. 2.4 gives 10th order in space);
 *   - a sponge absorbing layer padded outside the physical grid (Sec. 2.4 cites a
 *     sponge; profile and placement are readings, see below);
 *   - bi/tri-linear point sources and receivers (Sec. 2.4, off-grid sources and
 *     receivers by linear interpolation); injection is the transpose of sampling
 *     divided by the cell volume;
 *   - the exact discrete adjoint of that scheme, and the gradient of the L2 trace
 *     misfit with respect to vp by the adjoint-state method (Sec. 2.2, reduced
 *     objective and adjoint PDE; Sec. 3.2 describes one shot gradient as one
 *     forward and one adjoint propagation).
 *
 * Readings where the paper is silent (each is restated in the design notes):
 *   time order 2 (leapfrog); sponge outside the stated grid: a damping term
 *   eta dp/dt / vp^2 with eta = sum_axes eta_max_axis (d/nb)^2, d the depth in
 *   cells, and eta_max_axis = 3 vref ln(1/R0) / (nb dx_axis), so that the
 *   round-trip amplitude decay exp(-int eta/vref dx) through the layer is
 *   R0 = 1e-3; vref fixed per solve, so eta does not depend on vp
 *   (vref = 0 switches damping off but keeps the padding); vp edge-replicated
 *   into the layer; zero field beyond the padded array; traces[r][n] = R u^n with
 *   t_n = n dt; s^n drives u^{n+1}; misfit J = 1/2 sum (traces - observed)^2.
 *
 * Layout: C order, last axis contiguous.  Physical arrays have shape `shape`;
 * coordinates are metres with the origin at physical node 0, xyz[p*ndim + axis].
 * Traces and wavelets are [count][nt].
 *
 * Return codes: 0 ok, -1 bad argument, -3 a point lies outside the physical grid,
 * -7 out of host memory.
 */
#ifndef STRIDE_ORACLE_H
#define STRIDE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int ndim;            /* 2 or 3 */
    long shape[3];       /* physical grid */
    double spacing[3];   /* metres */
    int space_order;     /* 2, 4, 6, 8 or 10 */
    int nb;              /* sponge cells added on every side */
    double vref;         /* sponge reference speed (m/s); 0 = no damping */
    double dt;           /* seconds */
    int nt;              /* number of time samples */
    int time_order;      /* 2 (leapfrog) or 4 (leapfrog with the modified-equation
                            correction); 0 means 2 */
    int interp;          /* off-grid points: 0 bi/tri-linear, 1 Kaiser-windowed sinc */
} oracle_grid_t;

/* Windowed-sinc taps (Sec. 2.4 cites Hicks' Kaiser-windowed sinc functions for
 * off-grid sources and receivers): per axis the 2r nodes around the point,
 * weight sinc(x) I0(b sqrt(1 - (x/r)^2)) / I0(b) at offset x, the product over
 * the axes; a point on a node gets that node alone.  r = 4 and b = 6.31 are
 * readings (the window width and the Kaiser shape Hicks tabulates for it). */
#define ORACLE_SINC_HALF_WIDTH 4
#define ORACLE_SINC_KAISER_B 6.31

/* Central second-derivative weights c[0..order/2]. */
int oracle_fd_weights(int space_order, double *c);

/* Padded size per axis and total. */
long oracle_padded_points(const oracle_grid_t *g, long *npad3);

/* Edge-replicating pad of a physical field, and its transpose (sum of the
 * padded strips into the edge cells). */
int oracle_pad(const oracle_grid_t *g, const double *phys, double *pad);
int oracle_pad_transpose(const oracle_grid_t *g, const double *pad, double *phys);

/* Damping rate eta on the padded grid (1/s). */
int oracle_eta(const oracle_grid_t *g, double *eta);

/* Taps of npts points (linear or windowed sinc, per g->interp): T entries per
 * point (T = oracle_taps_per_point), idx[p*T+t] the padded linear index and
 * w[p*T+t] the weight, in C order over the per-axis node lists.  Each axis
 * lists the nodes closer than the reach (1 cell linear, 4 cells sinc), filled
 * up with weight-0 entries.  Returns -3 for a point outside the physical grid
 * or (sinc) whose window of 8 nodes per axis leaves the padded array. */
int oracle_taps(const oracle_grid_t *g, int npts, const double *xyz, long *idx, double *w);
/* Taps per point: 2^ndim (linear) or (2 r)^ndim (sinc); idx and w of
 * oracle_taps hold that many entries per point. */
int oracle_taps_per_point(const oracle_grid_t *g);

/* Apply the 2r-order Laplacian on the padded grid (zero outside). */
int oracle_laplacian(const oracle_grid_t *g, const double *u, double *lu);

/* Forward solve.  vp: physical [shape]; wavelet [nsrc][nt]; traces [nrec][nt].
 * nsnap > 0 stores u^n for n = snap_steps[i] into snaps[i][padded].
 *
 * time_order 4 (the paper's solver is fourth-order accurate in time, Sec. 2.4):
 * the leapfrog truncation error dt^2/12 u_tttt is cancelled by adding
 * dt^4/12 u_tttt with u_tttt = v^2 (L (v^2 (L u + S)) + S_tt) and
 * S_tt = (S^{n+1} - 2 S^n + S^{n-1}) / dt^2 (S^{-1} = 0).  With k = dt^2 v^2:
 *   p       = k (L u^n + St^n),   St^n = (S^{n-1} + 10 S^n + S^{n+1}) / 12
 *   u^{n+1} = a (2 u^n + p + (k/12) L p) - b u^{n-1}
 * (p is zero beyond the padded array, like u).
 *
 * Its exact discrete adjoint (T = K + (1/12) K L K is symmetric, K = diag k;
 * with w = K A lambda, A = diag a):
 *   q   = k L w^{m+1}
 *   w^m = a (2 w^{m+1} + q + (k/12) L q + k R^T g^m) - b w^{m+2}
 * and k dJ/dk sums w^{m+1} (v + (1/12) L p) + (1/12) q v with v = L u^m + St^m,
 * p = k v; dJ/dvp = P^T (2 G / vp) as in second order.  The wavelet
 * cotangent: dJ/dSt^m = w^{m+1} + q/12 sampled with the source taps / cell
 * volume, then the transpose of the time filter, (h^{j-1} + 10 h^j + h^{j+1}) / 12. */
int oracle_forward(const oracle_grid_t *g, const double *vp,
                   int nsrc, const double *src_xyz, const double *wavelet,
                   int nrec, const double *rec_xyz, double *traces,
                   int nsnap, const int *snap_steps, double *snaps);

/* Vector-Jacobian product of the forward map (vp, wavelet) -> traces, evaluated
 * at (vp, wavelet) with trace cotangent grad_traces [nrec][nt].  Outputs:
 * dvp (physical shape, may be NULL) and dwavelet [nsrc][nt] (may be NULL).
 * The forward states are kept by two-level checkpointing every `seg` steps
 * (seg <= 0 picks ceil(sqrt(nt))); the result does not depend on seg. */
int oracle_adjoint(const oracle_grid_t *g, const double *vp,
                   int nsrc, const double *src_xyz, const double *wavelet,
                   int nrec, const double *rec_xyz, const double *grad_traces,
                   double *dvp, double *dwavelet, int seg);

/* Shot gradient: traces (optional out), misfit J = 1/2 sum (traces-observed)^2
 * and dJ/dvp. */
int oracle_gradient(const oracle_grid_t *g, const double *vp,
                    int nsrc, const double *src_xyz, const double *wavelet,
                    int nrec, const double *rec_xyz, const double *observed,
                    double *traces_out, double *misfit, double *dvp, int seg);

/* Centred first-derivative weights d[1..r] of the (2r+1)-point antisymmetric
 * stencil exact on polynomials of degree <= 2r: du/dx ~ sum_j d_j (u_{+j} - u_{-j}) / dx. */
int oracle_fd1_weights(int space_order, double *d);

/* Heterogeneous medium (Sec. 2.4 acoustic equation with variable density and
 * power-law attenuation of exponent y = 0 or 2):
 *   (1/vp^2) p_tt = rho div(rho^{-1} grad p) + eta d/dt (-lap)^{y/2} p + s,
 *   eta = -2 alpha0 vp^{y-1}.
 * Discretisation (readings):
 *   rho div(rho^{-1} grad p) = lap p - grad(ln rho) . grad p, written
 *     L u + sum_a gamma_a D_a u with gamma_a = -D_a ln(rho_pad) and D_a the
 *     centred first derivative of the stencil's order; rho is edge-replicated
 *     into the sponge like vp, and ln rho beyond the padded array repeats its
 *     edge value (so gamma is the derivative of a field that is constant outward);
 *   y = 0: the term is -2 alpha0 vp^{-1} p_t, a damping that adds 2 alpha0 vp to
 *     the sponge's eta in the same centred form (a, b);
 *   y = 2: the term is 2 alpha0 vp dt(lap p); with k = dt^2 vp^2 it enters the
 *     update as k beta (L u^n - L u^{n-1}), beta = 2 alpha0 vp / dt (a backward
 *     difference, which keeps the step explicit);
 *   u^{n+1} = a (2 u^n + k (L u^n + sum_a gamma_a D_a u^n + S^n [+ beta (L u^n - L u^{n-1})]))
 *             - b u^{n-1}.
 * alpha0 is in Np/m for y = 0 and Np/m/(rad/s)^2 for y = 2 (amplitude decay
 * exp(-alpha0 omega^y r)).  rho (NULL = 1) and alpha0 (NULL = 0) are physical
 * arrays; rho must be positive and alpha0 non-negative.  Second-order time only
 * (time_order 4 returns -1), forward only. */
int oracle_medium_operator(const oracle_grid_t *g, const double *rho, const double *u,
                           double *out);
int oracle_forward_medium(const oracle_grid_t *g, const double *vp, const double *rho,
                          const double *alpha0, int att_power,
                          int nsrc, const double *src_xyz, const double *wavelet,
                          int nrec, const double *rec_xyz, double *traces);

/* Forward solve with a perfectly matched layer instead of the sponge (Sec. 2.4
 * offers a PML beside the sponge; the paper cites an unsplit formulation
 * without printing it).  Reading: complex coordinate stretching of each axis,
 * d_a -> (1/s_a) d_a with s_a = 1 + zeta_a/(i omega), in the second-order
 * equation written per axis,
 *   (1/vp^2) u_tt = sum_a (1/s_a) d_a ((1/s_a) d_a u) + s,
 * with memory variables for the two stretched derivatives:
 *   (1/s_a) d_a u = d_a u - psi_a,        psi_a' = zeta_a (d_a u - psi_a),
 *   (1/s_a) d_a q = d_a q - chi_a,        chi_a' = zeta_a (d_a q - chi_a),
 *   q = d_a u - psi_a, so d_a q = d_aa u - d_a psi_a.
 * Discretisation: d_aa = the axis-a part of the 2r-order Laplacian, d_a = the
 * centred first derivative of the same order (zero beyond the padded array);
 * the relaxations are integrated exactly over a step with their drive held
 * (E = exp(-zeta dt)):
 *   chi_a^n     = E chi_a^{n-1} + (1 - E) (d_aa u^n - d_a psi_a^n),
 *   psi_a^{n+1} = E psi_a^n     + (1 - E) d_a u^n,
 *   u^{n+1}     = 2 u^n - u^{n-1} + k (sum_a (d_aa u^n - d_a psi_a^n - chi_a^n) + S^n),
 * zeta_a = zeta_max,a (d/nb)^2 in the nb-cell layer of axis a (d = cells into
 * it), zeta_max,a = 3 vref ln(1/R0) / (2 nb dx_a), R0 = ORACLE_PML_R0 (the
 * continuous layer's round-trip reflection at normal incidence).  Sources are
 * not stretched (they lie in the physical grid).  Second-order time, forward
 * only; vref = 0 or nb = 0 gives the plain leapfrog without damping. */
#define ORACLE_PML_R0 1e-3
int oracle_forward_pml(const oracle_grid_t *g, const double *vp, int nsrc, const double *src_xyz,
                       const double *wavelet, int nrec, const double *rec_xyz, double *traces);

/* Adjoint and shot gradient of oracle_forward_medium (rho and alpha0 fixed):
 * the exact discrete transpose of the medium step, with w = a k lambda,
 *   w^m = a (2 w^{m+1} + k (L y - sum_a D_a (gamma_a w^{m+1}) + R^T g^m)) - b w^{m+2},
 *   y = (1 + beta) w^{m+1} - beta w^{m+2}  (beta = 0 for y = 0),
 * dvp = P^T sum_n w^{n+1} [ (2/vp) v^n + (y = 2) (2 alpha0/dt) (L u^n - L u^{n-1})
 *                         + (y = 0) (dt alpha0 a / k) (2 u^{n-1} - 2 u^n - k v^n) ],
 * v^n the step's right-hand side (L u^n + sum_a gamma_a D_a u^n + S^n + beta (L u^n -
 * L u^{n-1})); dwavelet[s][n] = W_s w^{n+1} / cell volume.  Two-level
 * checkpointing with segments of seg steps (seg <= 0: sqrt(nt)). */
int oracle_adjoint_medium(const oracle_grid_t *g, const double *vp, const double *rho,
                          const double *alpha0, int att_power, int nsrc, const double *src_xyz,
                          const double *wavelet, int nrec, const double *rec_xyz,
                          const double *grad_traces, double *dvp, double *dwavelet, int seg);
int oracle_gradient_medium(const oracle_grid_t *g, const double *vp, const double *rho,
                           const double *alpha0, int att_power, int nsrc, const double *src_xyz,
                           const double *wavelet, int nrec, const double *rec_xyz,
                           const double *observed, double *traces_out, double *misfit, double *dvp,
                           int seg);

/* Zero-phase low-pass of [count][nt] signals sampled at dt (the band-limiting
 * of wavelets and traces per frequency block, Sec. 3.2): out = h * in with
 * zeros outside the record, where h is a Hann-windowed sinc of cutoff f_max,
 *   h_k = 2 f_max dt sinc(2 f_max k dt) (0.5 + 0.5 cos(pi k / (K + 1))),
 *   |k| <= K = ceil(2 / (f_max dt)) (two periods of the cutoff each side),
 * scaled so that sum_k h_k = 1.  Returns the number of taps K, or -1. */
int oracle_lowpass(const double *in, double *out, int count, int nt, double dt, double f_max);

/* Number of OpenMP threads the oracle will use, and a way to change it (for
 * timing; the results do not depend on it). */
int oracle_num_threads(void);
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
