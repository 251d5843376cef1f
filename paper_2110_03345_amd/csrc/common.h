// Internal definitions shared by the host code and the HIP kernels of the
// acoustic FWI library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stride {

constexpr int kMaxR = 5;        // stencil radius (10th order)
constexpr int kThreads = 256;   // 4 wave64 per block
constexpr int kTileX = 64;      // contiguous axis: one wave64 spans a tile row
constexpr int kSincHalfWidth = 4;   // windowed-sinc taps: 2 r nodes per axis

// Launch shapes of the step kernels: rows per thread x wave64s per block (the
// tile is 64 x rows * waves) and, in 3D, planes per block.  The fastest
// measured on 1104^2 and 316^3.  The 3D adjoint shape also serves every step
// with two stencil fields (adjoint, fourth-order adjoint correction, medium);
// the adjoint steps that image from a stored v (one stencil field) take a
// taller tile of their own, with the adjoint's chunk length.
constexpr int kRy2d = 4, kWaves2d = 4;
constexpr int kRy3dFwd = 4, kWaves3dFwd = 8, kZc3dFwd = 32;
constexpr int kRy3dAdj = 2, kWaves3dAdj = 4, kZc3dAdj = 16;
constexpr int kRy3dAdjV = 4, kWaves3dAdjV = 4;
constexpr int kPitchAlign = 16;     // row pitch of the fields, in floats (64 B)

// Padded grid as laid out in the workspace.  Axis nd-1 is contiguous.
// 2D: axis 0 = rows, axis 1 = columns.  3D: axis 0 is the marching axis.
struct Dims {
    int nd;
    int n[3];          // padded extent per axis (unused axes = 1)
    int phys[3];       // physical extent
    int nb;            // sponge cells per side
    long long st[3];   // element strides; st[nd-1] = 1
    long long total;   // elements in one field (with row pitch)
};

// Laplacian weights already divided by dx_axis^2 (rounded once from FP64);
// c0 is the summed centre weight over all axes.
struct StencilCoef {
    float c0;
    float c[3][kMaxR + 1];
    float d[3][kMaxR + 1];   // centred first-derivative weights / dx_axis (medium steps)
};

// Sponge: eta = sum_axes e[a] * depth_a^2, e[a] = eta_max_a / nb^2.
struct SpongeCoef {
    float e[3];
    float half_dt;
};

// Injection entries grouped by step-kernel block (a 2D tile, or a 3D tile
// over one chunk of planes) of the launch shape that uses the table.  Block b
// holds ent[ptr[b] .. ptr[b+1]); entry e adds w * sig[id][step] at its
// block-local point `local` = (plane in chunk * TY + tile row) * 64 + tile
// column.  A block's entries are sorted by point, in (point, tap) order
// within a point; the first entry of a point holds the number of entries of
// that point in `run`, the others 0.
struct TileEntry {
    int local;
    int run;
    int id;
    float w;
};

struct InjTable {
    const int* ptr;
    const TileEntry* ent;
};

// Point sampling: v = scale * sum_t w[r*ntap+t] * field[idx[r*ntap+t]], stored to
// out[r * out_stride + step] or, with accumulate, added to it.
struct SampleSet {
    int count;
    const long long* idx;
    const float* w;
    float* out;
    int out_stride;
    int ntap;         // taps per point: 2^ndim (linear) or (2 r)^ndim (windowed sinc)
    float scale;
    int accumulate;
};

// Threads that sample one point: one for up to 8 taps, a wave64 (lanes over
// the taps, then a wave reduction) for the windowed-sinc tap sets.
__host__ __device__ inline int sample_lanes(int ntap)
{
    return ntap > 8 ? 64 : 1;
}

struct StepParams {
    const float* A;   // stencil field: u^n (forward) or w^{m+1} (adjoint)
    const float* B;   // u^{n-1} or w^{m+2}
    float* C;         // result; may alias B
    const float* K;   // dt^2 vp^2
    const float* U;   // adjoint only: second stencil field (u^m; p in the correction)
    float* G;         // adjoint only: imaging accumulator
    const float* D;   // correction only: point field u^n (forward) or w^{m+1} (adjoint)
    int step;         // time index of the injected / sampled signals
    InjTable inj;     // injection into C: sources (forward), receivers (adjoint)
    const float* inj_sig;
    int inj_stride;
    InjTable img;     // adjoint only: source term S^m of the imaging condition
    const float* img_sig;
    int img_stride;
    SampleSet smp;    // sampling of A at `step`
    // medium steps only: gamma_a = -D_a ln rho per axis, and the attenuation
    // field (att_power 0: 2 alpha0 vp added to the damping; 2: beta = 2 alpha0 vp / dt)
    const float* gam[3];
    const float* att;
    int att_power;
    float* V;         // kStepV: L u^n + S^n out; kImageV: that of u^m in
    const float* V2;  // kImageV: that of u^{m+1} (NULL: one imaging term per step)
};

// One slot's step in a batched launch.
struct SlotStep {
    StepParams p;
    SpongeCoef sp;
    int active;
};

struct LaunchShape {
    int ty;               // tile rows (waves x rows per thread)
    int ry, waves;        // rows per thread, wave64s per block
    int tiles_x, tiles_y, tiles_xy;
    int zc, nzc;          // 3D: planes per block and number of z chunks
    int tile_blocks;      // logical tile blocks (before XCD padding)
    int tile_blocks_pad;  // rounded up to a multiple of 8 XCDs
};

// Rows per thread and waves per block of the step kernels for a dimension
// and direction (the tile is 64 x ry*waves).
void tile_shape(int nd, bool adjoint, int* ry, int* waves);
// Shape of the adjoint steps imaging from a stored v (kImageV, kAdjPlain).
void tile_shape_v(int nd, int* ry, int* waves);

// What a step launch computes.  Fourth-order time runs two launches per
// forward step and three per adjoint step (kPrep on u^m and on w^{m+1}, then
// the adjoint kCorrect).
enum StepMode {
    kStep = 0,    // C = a (2 A + k (L A + S)) - b B                 (leapfrog step)
    kPrep = 1,    // C = k (L A + St), St: source filtered in time   (p of the corrected step)
    kCorrect = 2, // C = a (2 D + A + (k/12) L A) - b B, A = p, D = u^n;
                  // adjoint: C = a (2 D + A + (k/12) L A + k R^T g) - b B with A = q,
                  // D = w^{m+1}, and G += U (D + A/12) + (k/12) D L U with U = p
    kMedium = 3,  // forward step in a heterogeneous medium, B a stencil field too:
                  // C = a (2 A + k (L A + sum_a gam_a D_a A + S [+ att (L A - L B)])) - b B,
                  // with att added to the damping instead when att_power is 0; with V
                  // given it also stores the imaging factor of the vp gradient there
    kStepV = 4,   // forward kStep that also stores V = L A + S (full-history gradients)
    kImageV = 5,  // adjoint kStep whose imaging reads V = L u^m + S^m instead of the
                  // stencil of u^m: G += A V, and with V2 the previous step's term as
                  // well, G = fma(A, V, fma(B, V2, G)) (B = w^{m+2})
    kAdjPlain = 6 // adjoint kStep without imaging (the step before a kImageV with V2)
};

// Perfectly matched layer: the memory-variable correction of one step, for
// the points of the padded layer (the plain leapfrog without damping has
// already written u^{n+1}; see stride_grid_t.boundary).
struct PmlParams {
    const float* u;          // u^n
    float* un;               // u^{n+1}: += k (sum_a (-D_a psi_a^n - chi_a^n))
    const float* k;
    const float* psi[3];     // psi_a^n
    float* psin[3];          // psi_a^{n+1}
    float* chi[3];           // chi_a^{n-1} -> chi_a^n (in place)
    float c0[3];             // second-derivative centre weight / dx_a^2 per axis
    float zmax[3];           // zeta_max per axis (1/s)
    float dt;
};

// One adjoint step of the heterogeneous-medium gradient (the exact transpose
// of kMedium): w^m = a (2 w^{m+1} + k (L y - sum_a D_a (gam_a w^{m+1}))) - b w^{m+2},
// y = (1 + beta) w^{m+1} - beta w^{m+2} (beta = att when att_power is 2, else 0;
// with att_power 0 att joins the damping), and G += w^{m+1} H.  The receiver
// residual is added afterwards by launch_inject_table.
struct MediumAdjParams {
    const float* w1;         // w^{m+1}
    const float* w2;         // w^{m+2}
    float* w0;               // w^m
    const float* k;
    const float* gam[3];
    const float* att;        // 2 alpha0 vp (att_power 0) or beta (2); NULL: none
    int att_power;
    const float* H;          // imaging factor of step m; NULL: no imaging
    float* G;
};

// Kernel launchers (stride_kernels.hip).
// max_sample_threads: the largest count * sample_lanes(ntap) over the slots.
void launch_step_batched(const Dims& d, int R, bool adjoint, int mode, const StencilCoef& cf,
                         const LaunchShape& ls, const SlotStep* table, int nslots,
                         int max_sample_threads, hipStream_t s);
void launch_accumulate(float* dst, const float* src, long long n, hipStream_t s);
void launch_step(const Dims& d, int R, bool adjoint, const StencilCoef& cf, const SpongeCoef& sp,
                 const LaunchShape& ls, const StepParams& p, hipStream_t s);
// Launches of the mode steps: forward kPrep, kCorrect, kMedium or kStepV; adjoint
// kCorrect or kImageV.
void launch_step_mode(const Dims& d, int R, bool adjoint, int mode, const StencilCoef& cf,
                      const SpongeCoef& sp, const LaunchShape& ls, const StepParams& p, hipStream_t s);

void launch_pml_correction(const Dims& d, int R, const StencilCoef& cf, const PmlParams& pp,
                           hipStream_t s);
void launch_medium_adjoint(const Dims& d, int R, const StencilCoef& cf, const SpongeCoef& sp,
                           const MediumAdjParams& mp, hipStream_t s);
// out[p] += a(p) k(p) (sum of the signals injected at p), for every point of an
// injection table built for the launch shape ls; a(p) the damping factor of
// the sponge and (att_power 0) the attenuation field att.
void launch_inject_table(const Dims& d, const LaunchShape& ls, const InjTable& T, const float* sig,
                         int stride, int step, const float* k, const float* att, int att_power,
                         const SpongeCoef& sp, float* out, hipStream_t s);
void launch_sample(const SampleSet& smp, const float* field, int step, hipStream_t s);
void launch_fill(float* p, long long n, float v, hipStream_t s);
// In place, per [nt] row: h[j] = (h[j-1] + 10 h[j] + h[j+1]) / 12 (zero outside),
// the transpose of the fourth-order scheme's source filter.
void launch_time_filter3(float* rows, int count, int nt, hipStream_t s);
// Zero-phase FIR low-pass of [count][nt] rows (out may alias in); K taps per side.
int lowpass_taps(double dt, double f_max);
void launch_lowpass(const float* in, float* out, int count, int nt, double dt, double f_max,
                    hipStream_t s);
// vp = clamp(vp - step m g / max|m g|, vmin, vmax); work: one device word.
void launch_descent(float* vp, const float* g, const float* mask, long long n, float step,
                    float vmin, float vmax, unsigned* work, hipStream_t s);
void launch_prep_k(const Dims& d, const float* vp, double dt, float* k, hipStream_t s);
// First-derivative weights in FP64 for the medium preparation.
struct Fd1 {
    double d[kMaxR + 1];
    double inv_dx[3];
    int r;
};

// Medium fields on the padded grid: gam[a] = -D_a ln rho_pad (rho NULL: zero;
// ln rho repeats its edge value beyond the array) and att (alpha0 NULL: zero;
// att_power 0: 2 alpha0 vp, 2: 2 alpha0 vp / dt), computed in FP64, rounded once.
void launch_prep_medium(const Dims& d, const Fd1& fd, const float* vp, const float* rho,
                        const float* alpha0, int att_power, double dt, float* const gam[3],
                        float* att, hipStream_t s);
// flags[2] = 1 if rho has a non-positive or non-finite value or alpha0 a negative
// or non-finite one; flags[3] = max over points of vp^2 (1 + 2 beta) as float bits
// (beta = 2 alpha0 vp / dt for att_power 2, else 0).
void launch_medium_check(const float* vp, const float* rho, const float* alpha0, long long n,
                         int att_power, double dt, unsigned* flags, hipStream_t s);
// Misfit partial sums: kMisfitParts doubles of scratch.
constexpr int kMisfitParts = 256;
void launch_residual_misfit(const float* traces, const float* observed, float* residual,
                            long long n, double* misfit, double* partial, hipStream_t s);
// dvp = P^T (2 G / vp_pad), with G = H / kdiv where kdiv is given (else G = H);
// tmp0 and tmp1 hold intermediates of up to one field each.
void launch_finalize_dvp(const Dims& d, const float* H, const float* kdiv, const float* vp,
                         float* dvp, float* tmp0, float* tmp1, hipStream_t s);
void launch_copy(float* dst, const float* src, long long n, hipStream_t s);
// *flag |= bit if any of the n values is NaN or infinite (flag cleared by the caller).
void launch_finite_scan(const float* p, long long n, unsigned* flag, unsigned bit, hipStream_t s);
void launch_finite_scan(const double* p, long long n, unsigned* flag, unsigned bit, hipStream_t s);
// flags[0] = bits of max(vp) (vp > 0), flags[1] = 1 if any vp <= 0 or non-finite.
void launch_vp_check(const float* vp, long long n, unsigned* flags, hipStream_t s);

}  // namespace stride
