// HIP kernels for gfx950 (CDNA4): leapfrog step of the acoustic wave
// equation with a 2r-order Laplacian and a sponge layer, fused with point
// injection, point sampling and (adjoint variant) the imaging condition.
//
// Forward (paper Sec. 2.4, constant density, no attenuation; second order in
// time):   C = a (2 A + k (L A + S)) - b B,          a = b = 1 outside the sponge
// Adjoint (exact transpose, Sec. 2.2 adjoint PDE):  the same update with
//          A = w^{m+1}, B = w^{m+2}, S = R^T g^m,  plus the imaging term
//          G += w^{m+1} (L u^m + S^m)   (gradient w.r.t. k; Sec. 2.2 reduced
//          gradient <grad_m L* w, dm>).
//
// The kernels are HBM-bound (16 B per forward update, 28 B per adjoint update):
// no MFMA.  Tiles are 64 wide along the contiguous axis (one wave64 per tile
// row, 256 B coalesced) and 16 rows high; the u^n tile plus its halo sits in
// LDS.  In 3D each block marches along axis 0 over a chunk of planes, keeping
// the 2r+1 values of its column in registers (2.5D blocking), so each plane of
// u^n is read once from HBM and the axis-0 neighbours never touch LDS.

//
// This file holds the small kernels and the launchers; the step kernels
// live in step_kernels.h and compile in their own translation units.
#include "step_kernels.h"

#include <algorithm>
#include <cstdlib>

namespace stride {

// Tile shapes the kernels use (the host sizes launch shapes with these): the
// constants of common.h.  A build with STRIDE_TILE_SWEEP compiles every shape
// the sweeps try and reads the choice from the environment (STRIDE_RY2D[_ADJ],
// STRIDE_WAVES2D[_ADJ], STRIDE_RY3D[_ADJ], STRIDE_WAVES3D[_ADJ]); the library
// as shipped ignores the environment.
void tile_shape(int nd, bool adjoint, int* ry, int* waves)
{
#ifdef STRIDE_TILE_SWEEP
    if (nd == 2) {
        const char* er = getenv(adjoint ? "STRIDE_RY2D_ADJ" : "STRIDE_RY2D");
        const char* ew = getenv(adjoint ? "STRIDE_WAVES2D_ADJ" : "STRIDE_WAVES2D");
        int r = er && *er ? atoi(er) : kRy2d;
        int w = ew && *ew ? atoi(ew) : kWaves2d;
        if (w == 8) {
            r = 4;
        } else {
            w = 4;
            if (r != 2 && r != 8)
                r = 4;
        }
        *ry = r;
        *waves = w;
        return;
    }
    const char* er = getenv(adjoint ? "STRIDE_RY3D_ADJ" : "STRIDE_RY3D");
    const char* ew = getenv(adjoint ? "STRIDE_WAVES3D_ADJ" : "STRIDE_WAVES3D");
    int r = er && *er ? atoi(er) : (adjoint ? kRy3dAdj : kRy3dFwd);
    int w = ew && *ew ? atoi(ew) : (adjoint ? kWaves3dAdj : kWaves3dFwd);
    if (w != 8)
        w = 4;
    if (r != 1 && r != 2)
        r = 4;
    if (w == 4 && r == 1)
        r = 2;
    *ry = r;
    *waves = w;
#else
    if (nd == 2) {
        *ry = kRy2d;
        *waves = kWaves2d;
    } else {
        *ry = adjoint ? kRy3dAdj : kRy3dFwd;
        *waves = adjoint ? kWaves3dAdj : kWaves3dFwd;
    }
#endif
}

void tile_shape_v(int nd, int* ry, int* waves)
{
    if (nd == 2) {
        tile_shape(nd, true, ry, waves);
        return;
    }
#ifdef STRIDE_TILE_SWEEP
    const char* er = getenv("STRIDE_RY3D_ADJV");
    const char* ew = getenv("STRIDE_WAVES3D_ADJV");
    int r = er && *er ? atoi(er) : kRy3dAdjV;
    int w = ew && *ew ? atoi(ew) : kWaves3dAdjV;
    if (w != 8)
        w = 4;
    if (r != 1 && r != 2)
        r = 4;
    if (w == 4 && r == 1)
        r = 2;
    *ry = r;
    *waves = w;
#else
    *ry = kRy3dAdjV;
    *waves = kWaves3dAdjV;
#endif
}

namespace {

// ------------------------------------------------------------ small kernels

__global__ void sample_kernel(SampleSet smp, const float* field, int step)
{
    sample_block(smp, field, step, blockIdx.x);
}

__global__ void fill_kernel(float* p, long long n, float v)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

__global__ void copy_kernel(float* dst, const float* src, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        dst[i] = src[i];
}

// k = dt^2 vp_pad^2 with vp edge-replicated into the sponge; computed in
// double and rounded once.
__global__ void prep_k_kernel(Dims d, const float* vp, double dt, float* k)
{
    long long npts = (long long)d.n[0] * d.n[1] * d.n[2];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < npts; i += stride) {
        int c[3];
        long long r = i;
        for (int a = 2; a >= 0; --a) {
            c[a] = (int)(r % d.n[a]);
            r /= d.n[a];
        }
        long long src = 0, dst = 0;
        for (int a = 0; a < 3; ++a) {
            int pa = min(max(c[a] - d.nb, 0), d.phys[a] - 1);
            if (d.n[a] == 1)
                pa = 0;
            src = src * d.phys[a] + pa;
            dst += (long long)c[a] * (a < d.nd ? d.st[a] : 0);
        }
        double v = (double)vp[src];
        k[dst] = (float)(dt * dt * v * v);
    }
}

// Medium fields on the padded grid (see launch_prep_medium).  The physical
// index of any padded (or beyond-padded) coordinate is its clamp into the
// physical grid, which is both the edge replication into the sponge and the
// constant continuation of ln rho beyond the array.
__device__ __forceinline__ long long phys_index(const Dims& d, const int c[3])
{
    long long src = 0;
    for (int a = 0; a < 3; ++a) {
        int pa = a < d.nd ? min(max(c[a] - d.nb, 0), d.phys[a] - 1) : 0;
        src = src * d.phys[a] + pa;
    }
    return src;
}

__global__ void prep_medium_kernel(Dims d, Fd1 fd, const float* vp, const float* rho,
                                   const float* alpha0, int att_power, double dt, float* g0,
                                   float* g1, float* g2, float* att)
{
    const long long npts = (long long)d.n[0] * d.n[1] * d.n[2];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    float* gam[3] = {g0, g1, g2};
    for (; i < npts; i += stride) {
        int c[3];
        long long r = i;
        for (int a = 2; a >= 0; --a) {
            c[a] = (int)(r % d.n[a]);
            r /= d.n[a];
        }
        long long dst = 0;
        for (int a = 0; a < d.nd; ++a)
            dst += (long long)c[a] * d.st[a];
        const long long src = phys_index(d, c);
        for (int a = 0; a < d.nd; ++a) {
            double sum = 0.0;
            if (rho) {
                for (int j = 1; j <= fd.r; ++j) {
                    int cp[3] = {c[0], c[1], c[2]}, cm[3] = {c[0], c[1], c[2]};
                    cp[a] += j;
                    cm[a] -= j;
                    sum += fd.d[j] * (log((double)rho[phys_index(d, cp)]) -
                                      log((double)rho[phys_index(d, cm)]));
                }
            }
            gam[a][dst] = (float)(-sum * fd.inv_dx[a]);
        }
        double at = 0.0;
        if (alpha0) {
            at = 2.0 * (double)alpha0[src] * (double)vp[src];
            if (att_power == 2)
                at /= dt;
        }
        att[dst] = (float)at;
    }
}

// Value checks of rho and alpha0, and max vp^2 (1 + 2 beta) for the stability
// limit of the y = 2 term (see launch_medium_check).
__global__ void medium_check_kernel(const float* vp, const float* rho, const float* alpha0,
                                    long long n, int att_power, double dt, unsigned* flags)
{
    __shared__ unsigned smax, sbad;
    if (threadIdx.x == 0) {
        smax = 0u;
        sbad = 0u;
    }
    __syncthreads();
    unsigned m = 0u, bad = 0u;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        if (rho && !(rho[i] > 0.f && isfinite(rho[i])))
            bad = 1u;
        double beta = 0.0;
        if (alpha0) {
            const float al = alpha0[i];
            if (!(al >= 0.f && isfinite(al)))
                bad = 1u;
            else if (att_power == 2)
                beta = 2.0 * (double)al * (double)vp[i] / dt;
        }
        const double v = (double)vp[i];
        const float e = (float)(v * v * (1.0 + 2.0 * beta));
        if (e >= 0.f && isfinite(e))
            m = max(m, __float_as_uint(e));
        else
            bad = 1u;
    }
    atomicMax(&smax, m);
    atomicOr(&sbad, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(&flags[3], smax);
        atomicOr(&flags[2], sbad);
    }
}

// Transposed source filter of the fourth-order scheme, one row per block,
// in place (the row is staged in LDS first).
__global__ __launch_bounds__(256) void time_filter3_kernel(float* rows, int nt)
{
    extern __shared__ float row[];
    float* r = rows + (long long)blockIdx.x * nt;
    for (int j = threadIdx.x; j < nt; j += 256)
        row[j] = r[j];
    __syncthreads();
    for (int j = threadIdx.x; j < nt; j += 256) {
        const float lo = j >= 1 ? row[j - 1] : 0.f;
        const float hi = j + 1 < nt ? row[j + 1] : 0.f;
        r[j] = fmaf(10.f, row[j], lo + hi) / 12.f;
    }
}

// Zero-phase low-pass of one [nt] row per block (band-limiting for the
// frequency blocks of an inversion): the Hann-windowed sinc taps
// h_k = 2 fc dt sinc(2 fc k dt) (0.5 + 0.5 cos(pi k / (K + 1))), |k| <= K,
// normalised to unit sum, are built in LDS (FP64, rounded once), the row is
// staged in LDS (so out may alias in), and each thread convolves its samples
// with zeros beyond the record.
__global__ __launch_bounds__(256) void lowpass_kernel(const float* in, float* out, int nt,
                                                      double fdt, int K)
{
    extern __shared__ float lds[];
    float* h = lds;                  // 2K + 1 taps
    float* row = lds + 2 * K + 1;    // nt samples
    __shared__ double part[256];
    const double pi = 3.14159265358979323846;
    double sum = 0.0;
    for (int k = -K + (int)threadIdx.x; k <= K; k += 256) {
        const double x = 2.0 * fdt * k;
        const double sc = k == 0 ? 1.0 : sin(pi * x) / (pi * x);
        const double v = 2.0 * fdt * sc * (0.5 + 0.5 * cos(pi * k / (K + 1.0)));
        sum += v;
    }
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double total = part[0];
    for (int k = -K + (int)threadIdx.x; k <= K; k += 256) {
        const double x = 2.0 * fdt * k;
        const double sc = k == 0 ? 1.0 : sin(pi * x) / (pi * x);
        h[k + K] = (float)(2.0 * fdt * sc * (0.5 + 0.5 * cos(pi * k / (K + 1.0))) / total);
    }
    const float* src = in + (long long)blockIdx.x * nt;
    for (int n = threadIdx.x; n < nt; n += 256)
        row[n] = src[n];
    __syncthreads();
    float* dst = out + (long long)blockIdx.x * nt;
    for (int n = threadIdx.x; n < nt; n += 256) {
        const int klo = max(-K, n - nt + 1), khi = min(K, n);
        float acc = 0.f;
        for (int k = klo; k <= khi; ++k)
            acc = fmaf(h[k + K], row[n - k], acc);
        dst[n] = acc;
    }
}

// Gradient-descent step of the inversion loop: gmax = max |m g| (as float
// bits; order-independent, so reproducible), then vp = clamp(vp - step m g /
// gmax, vmin, vmax) with the mask m (1 where absent).
__global__ __launch_bounds__(256) void grad_absmax_kernel(const float* g, const float* mask,
                                                          long long n, unsigned* gmax)
{
    __shared__ unsigned smax;
    if (threadIdx.x == 0)
        smax = 0u;
    __syncthreads();
    unsigned m = 0u;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float v = fabsf(mask ? mask[i] * g[i] : g[i]);
        m = max(m, __float_as_uint(v));
    }
    atomicMax(&smax, m);
    __syncthreads();
    if (threadIdx.x == 0)
        atomicMax(gmax, smax);
}

__global__ void descent_kernel(float* vp, const float* g, const float* mask, long long n,
                               float step, float vmin, float vmax, const unsigned* gmax)
{
    const float gm = __uint_as_float(*gmax);
    const float scale = gm > 0.f ? step / gm : 0.f;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float d = mask ? mask[i] * g[i] : g[i];
        vp[i] = fminf(fmaxf(fmaf(-scale, d, vp[i]), vmin), vmax);
    }
}

// Residual r = traces - observed and J = 1/2 sum r^2 in FP64.  Block b reduces
// a fixed contiguous range in a fixed tree order and misfit_final_kernel adds
// the partial sums in block order, so the result is bitwise reproducible.
__global__ __launch_bounds__(256) void residual_partial_kernel(const float* traces,
                                                               const float* observed,
                                                               float* residual, long long n,
                                                               double* partial)
{
    __shared__ double part[256];
    const long long per = (n + gridDim.x - 1) / gridDim.x;
    const long long lo = per * blockIdx.x;
    const long long hi = min(n, lo + per);
    double acc = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += 256) {
        float r = traces[i] - observed[i];
        residual[i] = r;
        acc += (double)r * (double)r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partial[blockIdx.x] = part[0];
}

__global__ __launch_bounds__(256) void misfit_final_kernel(const double* partial, int nparts,
                                                           double* misfit)
{
    __shared__ double part[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256)
        acc += partial[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *misfit = 0.5 * part[0];
}

// Transpose of edge-replicating padding along one axis.  The input is viewed
// as [m0][nin][m2] with strides (s_outer, s_axis, 1), the output is dense
// [m0][nout][m2] with nin = nout + 2 nb: output cell j collects input cell
// j + nb, and the two edge cells also collect the nb cells replicated from
// them.  With vp given, the output is 2 * sum / vp (the last pass of dvp).
// With div given (laid out like the input), each input cell is divided by it.
__global__ void pad_transpose_axis_kernel(const float* in, const float* div, long long s_outer,
                                          long long s_axis, float* out, long long m0, int nout,
                                          long long m2, int nb, const float* vp)
{
    const long long total = m0 * nout * m2;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < total; i += stride) {
        const long long i2 = i % m2;
        const long long r = i / m2;
        const int j = (int)(r % nout);
        const long long i0 = r / nout;
        const int lo = j == 0 ? 0 : j + nb;
        const int hi = j == nout - 1 ? j + 2 * nb : j + nb;
        const long long base = i0 * s_outer + i2;
        const float* src = in + base;
        float acc = 0.f;
        if (div)
            for (int k = lo; k <= hi; ++k)
                acc += src[(long long)k * s_axis] / div[base + (long long)k * s_axis];
        else
            for (int k = lo; k <= hi; ++k)
                acc += src[(long long)k * s_axis];
        out[i] = vp ? 2.f * acc / vp[i] : acc;
    }
}

// max(vp) (as the bit pattern of a positive float, which orders like the
// float) and a flag for non-positive or non-finite values.
__global__ void vp_check_kernel(const float* vp, long long n, unsigned* flags)
{
    __shared__ unsigned smax, sbad;
    if (threadIdx.x == 0) {
        smax = 0u;
        sbad = 0u;
    }
    __syncthreads();
    unsigned m = 0u, bad = 0u;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        float v = vp[i];
        if (!(v > 0.f) || !isfinite(v))
            bad = 1u;
        else
            m = max(m, __float_as_uint(v));
    }
    atomicMax(&smax, m);
    atomicOr(&sbad, bad);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(&flags[0], smax);
        atomicOr(&flags[1], sbad);
    }
}

int grid_for(long long n, int threads)
{
    long long b = (n + threads - 1) / threads;
    if (b > 65536)
        b = 65536;
    if (b < 1)
        b = 1;
    return (int)b;
}

}  // namespace


// Step launches go to the translation unit of their family.
void launch_family_2d(bool adjoint, int R, int mode, const Dims& d, const StencilCoef& cf,
                      const SpongeCoef& sp, const LaunchShape& ls, const StepParams& p, hipStream_t s);
void launch_family_3d_fwd(int R, int mode, const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                          const LaunchShape& ls, const StepParams& p, hipStream_t s);
void launch_family_3d_adj(int R, int mode, const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                          const LaunchShape& ls, const StepParams& p, hipStream_t s);
void launch_batched_2d(bool adjoint, int R, int mode, const Dims& d, const StencilCoef& cf,
                       const LaunchShape& ls, const SlotStep* table, int nslots, int max_samples,
                       hipStream_t s);
void launch_batched_3d_fwd(int R, int mode, const Dims& d, const StencilCoef& cf,
                           const LaunchShape& ls, const SlotStep* table, int nslots, int max_samples,
                           hipStream_t s);
void launch_batched_3d_adj(int R, int mode, const Dims& d, const StencilCoef& cf,
                           const LaunchShape& ls, const SlotStep* table, int nslots, int max_samples,
                           hipStream_t s);

void launch_step_mode(const Dims& d, int R, bool adjoint, int mode, const StencilCoef& cf,
                      const SpongeCoef& sp, const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    if (d.nd == 2)
        launch_family_2d(adjoint, R, mode, d, cf, sp, ls, p, s);
    else if (adjoint)
        launch_family_3d_adj(R, mode, d, cf, sp, ls, p, s);
    else
        launch_family_3d_fwd(R, mode, d, cf, sp, ls, p, s);
}

void launch_step(const Dims& d, int R, bool adjoint, const StencilCoef& cf, const SpongeCoef& sp,
                 const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    launch_step_mode(d, R, adjoint, kStep, cf, sp, ls, p, s);
}

void launch_step_batched(const Dims& d, int R, bool adjoint, int mode, const StencilCoef& cf,
                         const LaunchShape& ls, const SlotStep* table, int nslots, int max_samples,
                         hipStream_t s)
{
    if (d.nd == 2)
        launch_batched_2d(adjoint, R, mode, d, cf, ls, table, nslots, max_samples, s);
    else if (adjoint)
        launch_batched_3d_adj(R, mode, d, cf, ls, table, nslots, max_samples, s);
    else
        launch_batched_3d_fwd(R, mode, d, cf, ls, table, nslots, max_samples, s);
}

__global__ void accumulate_kernel(float* dst, const float* src, long long n)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        dst[i] += src[i];
}

void launch_accumulate(float* dst, const float* src, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(accumulate_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
}

void launch_sample(const SampleSet& smp, const float* field, int step, hipStream_t s)
{
    if (smp.count <= 0)
        return;
    int blocks = (smp.count * sample_lanes(smp.ntap) + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(sample_kernel, dim3(blocks), dim3(kThreads), 0, s, smp, field, step);
}

void launch_fill(float* p, long long n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
}

void launch_copy(float* dst, const float* src, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
}

// flag |= bit when any of the n values is NaN or infinite.
template <class T>
__global__ void finite_scan_kernel(const T* p, long long n, unsigned* flag, unsigned bit)
{
    bool bad = false;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        bad |= !isfinite(p[i]);
    if (bad)
        atomicOr(flag, bit);
}

void launch_finite_scan(const float* p, long long n, unsigned* flag, unsigned bit, hipStream_t s)
{
    hipLaunchKernelGGL(finite_scan_kernel<float>, dim3(std::min(grid_for(n, 256), 2048)), dim3(256),
                       0, s, p, n, flag, bit);
}

void launch_finite_scan(const double* p, long long n, unsigned* flag, unsigned bit, hipStream_t s)
{
    hipLaunchKernelGGL(finite_scan_kernel<double>, dim3(std::min(grid_for(n, 256), 2048)), dim3(256),
                       0, s, p, n, flag, bit);
}

// Perfectly matched layer.  Per axis a whose layer holds a point (zeta_a > 0):
//   chi_a = E chi_a + (1 - E) (D2_a u - D_a psi_a),  psi_a' = E psi_a + (1 - E) D_a u,
// and u^{n+1} += k sum_a (-D_a psi_a - chi_a), the axes taken in order 0, 1, 2.
// Neighbours beyond the padded array read 0.  One thread per point of the
// layer, over three launches of 64-lane rows (no index division): the planes
// of axis 0 in its layer (3D), then within the physical planes the rows of
// axis 1 in its layer, then within the physical rows the points of axis 2 in
// its layer.  Blocks are 4 rows; in the first launch the rows of a block are 4
// consecutive planes and consecutive blocks continue along axis 0, so the 2R
// axis-0 neighbours a point reads come from the same or a neighbouring block
// (L2) rather than from a plane's distance away in the launch.
struct PmlGeom {
    int nn[3];        // 3D-ised padded extents (axis 0 of a 2D grid has extent 1)
    int st[3];        // strides in floats (pitched rows)
    int pl[3];        // physical extents
    int b;            // layer width of axes 1 and 2 (and of axis 0 in 3D)
    int b0;           // layer width of axis 0 (0 in 2D)
    int three;
};

template <int R>
__device__ __forceinline__ void pml_axis_term(const StencilCoef& cf, const PmlParams& pp,
                                              const PmlGeom& g, long long p, const int* ii, int ax,
                                              float& corr)
{
    const int a = g.three ? ax : ax - 1;        // axis of the solver's Dims / coefficients
    const int i = ii[ax];
    const int b = ax == 0 ? g.b0 : g.b;
    const int hi = b + g.pl[ax] - 1;
    const int depth = i < b ? b - i : (i > hi ? i - hi : 0);
    if (depth == 0)
        return;
    const float frac = (float)depth / (float)b;
    const float zeta = pp.zmax[a] * frac * frac;
    const float E = __expf(-zeta * pp.dt);   // hardware exp2: a few ulp, far inside the tolerance
    const float* u = pp.u + p;
    const float* psi = pp.psi[a] + p;
    const int s = g.st[ax];
    float d2 = pp.c0[a] * u[0], d1u = 0.f, d1p = 0.f;
#pragma unroll
    for (int j = 1; j <= R; ++j) {
        const bool in_p = i + j < g.nn[ax], in_m = i - j >= 0;
        const float up = in_p ? u[j * s] : 0.f;
        const float um = in_m ? u[-j * s] : 0.f;
        const float qp = in_p ? psi[j * s] : 0.f;
        const float qm = in_m ? psi[-j * s] : 0.f;
        d2 = fmaf(cf.c[a][j], up + um, d2);
        d1u = fmaf(cf.d[a][j], up - um, d1u);
        d1p = fmaf(cf.d[a][j], qp - qm, d1p);
    }
    const float chi = fmaf(E, pp.chi[a][p], (1.f - E) * (d2 - d1p));
    pp.chi[a][p] = chi;
    pp.psin[a][p] = fmaf(E, psi[0], (1.f - E) * d1u);
    corr -= d1p + chi;
}

template <int R>
__device__ __forceinline__ void pml_point(const StencilCoef& cf, const PmlParams& pp, const PmlGeom& g,
                                          int i0, int i1, int i2)
{
    const int ii[3] = {i0, i1, i2};
    const long long p = (long long)i0 * g.st[0] + (long long)i1 * g.st[1] + i2;
    float corr = 0.f;
    for (int ax = g.three ? 0 : 1; ax < 3; ++ax)
        pml_axis_term<R>(cf, pp, g, p, ii, ax, corr);
    pp.un[p] = fmaf(pp.k[p], corr, pp.un[p]);
}

// Planes of axis 0 in its layer: grid (2 ceil(b0/4), column chunks, rows);
// blockIdx.x = side x plane group (fastest), wave = plane within the group.
template <int R>
__global__ __launch_bounds__(256) void pml_layer0_kernel(Dims d, StencilCoef cf, PmlParams pp,
                                                         PmlGeom g)
{
    const int groups = (g.b0 + 3) / 4;
    const int side = (int)blockIdx.x >= groups;
    const int zl = ((int)blockIdx.x - side * groups) * 4 + ((int)threadIdx.x >> 6);
    const int i2 = (int)blockIdx.y * 64 + ((int)threadIdx.x & 63);
    if (zl >= g.b0 || i2 >= g.nn[2])
        return;
    const int i0 = side == 0 ? zl : g.b0 + g.pl[0] + zl;
    pml_point<R>(cf, pp, g, i0, (int)blockIdx.z, i2);
}

// Rows of axis 1 in its layer, in the physical planes: grid (column chunks,
// ceil(2b/4), physical planes).
template <int R>
__global__ __launch_bounds__(256) void pml_layer1_kernel(Dims d, StencilCoef cf, PmlParams pp,
                                                         PmlGeom g)
{
    const int rl = (int)blockIdx.y * 4 + ((int)threadIdx.x >> 6);
    const int i2 = (int)blockIdx.x * 64 + ((int)threadIdx.x & 63);
    if (rl >= 2 * g.b || i2 >= g.nn[2])
        return;
    const int i1 = rl < g.b ? rl : g.b + g.pl[1] + (rl - g.b);
    pml_point<R>(cf, pp, g, g.b0 + (int)blockIdx.z, i1, i2);
}

// Points of axis 2 in its layer, in the physical rows of the physical planes:
// one 64-lane row per (plane, row) with lanes 0 .. 2b-1 on the layer's points
// (b <= 32; wider layers take several lane groups); grid (lane groups x
// ceil(rows/4), physical planes).
template <int R>
__global__ __launch_bounds__(256) void pml_layer2_kernel(Dims d, StencilCoef cf, PmlParams pp,
                                                         PmlGeom g)
{
    const int lanes = (2 * g.b + 63) / 64;      // 64-lane groups per row
    const int rg = (int)blockIdx.x / lanes;
    const int lg = (int)blockIdx.x - rg * lanes;
    const int yi = rg * 4 + ((int)threadIdx.x >> 6);
    const int xl = lg * 64 + ((int)threadIdx.x & 63);
    if (yi >= g.pl[1] || xl >= 2 * g.b)
        return;
    const int i2 = xl < g.b ? xl : g.b + g.pl[2] + (xl - g.b);
    pml_point<R>(cf, pp, g, g.b0 + (int)blockIdx.y, g.b + yi, i2);
}

void launch_pml_correction(const Dims& d, int R, const StencilCoef& cf, const PmlParams& pp,
                           hipStream_t s)
{
    const bool three = d.nd == 3;
    PmlGeom g{};
    g.three = three ? 1 : 0;
    g.nn[0] = three ? d.n[0] : 1;
    g.nn[1] = three ? d.n[1] : d.n[0];
    g.nn[2] = three ? d.n[2] : d.n[1];
    g.st[0] = three ? (int)d.st[0] : 0;
    g.st[1] = three ? (int)d.st[1] : (int)d.st[0];
    g.st[2] = 1;
    g.pl[0] = three ? d.phys[0] : 1;
    g.pl[1] = three ? d.phys[1] : d.phys[0];
    g.pl[2] = three ? d.phys[2] : d.phys[1];
    g.b = d.nb;
    g.b0 = three ? d.nb : 0;
    if (g.b <= 0)
        return;
    const unsigned cch = (unsigned)((g.nn[2] + 63) / 64);
    const unsigned lanes = (unsigned)((2 * g.b + 63) / 64);
    const dim3 g0(2 * ((g.b0 + 3) / 4), cch, g.nn[1]);
    const dim3 g1(cch, (2 * g.b + 3) / 4, g.pl[0]);
    const dim3 g2(lanes * ((g.pl[1] + 3) / 4), g.pl[0]);
    if (R == 4) {
        if (g.b0 > 0)
            hipLaunchKernelGGL(pml_layer0_kernel<4>, g0, dim3(256), 0, s, d, cf, pp, g);
        hipLaunchKernelGGL(pml_layer1_kernel<4>, g1, dim3(256), 0, s, d, cf, pp, g);
        hipLaunchKernelGGL(pml_layer2_kernel<4>, g2, dim3(256), 0, s, d, cf, pp, g);
    } else {
        if (g.b0 > 0)
            hipLaunchKernelGGL(pml_layer0_kernel<5>, g0, dim3(256), 0, s, d, cf, pp, g);
        hipLaunchKernelGGL(pml_layer1_kernel<5>, g1, dim3(256), 0, s, d, cf, pp, g);
        hipLaunchKernelGGL(pml_layer2_kernel<5>, g2, dim3(256), 0, s, d, cf, pp, g);
    }
}

// Padded coordinates of linear index t over the padded grid (no pitch) and the
// sponge rate there.
__device__ __forceinline__ void padded_coords(const Dims& d, long long t, int c[3])
{
    c[2] = 0;
    if (d.nd == 3) {
        const long long plane = (long long)d.n[1] * d.n[2];
        c[0] = (int)(t / plane);
        const long long r = t - (long long)c[0] * plane;
        c[1] = (int)(r / d.n[2]);
        c[2] = (int)(r - (long long)c[1] * d.n[2]);
    } else {
        c[0] = (int)(t / d.n[1]);
        c[1] = (int)(t - (long long)c[0] * d.n[1]);
    }
}

__device__ __forceinline__ float sponge_eta(const Dims& d, const SpongeCoef& sp, const int c[3])
{
    float eta = 0.f;
    for (int a = 0; a < d.nd; ++a) {
        const int dep = layer_depth(c[a], d.n[a], d.nb);
        eta = fmaf(sp.e[a], (float)(dep * dep), eta);
    }
    return eta;
}

// One thread per padded point of a 64 x 8 tile of the plane spanned by the
// last two axes (the row axis ay and the contiguous axis ax), one plane per
// block (3D: blockIdx.z), two rows per thread.  The block first stages in LDS
// the stencil operand y over the tile and its R-wide halo, and the density
// products gamma_ay w^{m+1} (tile and row halo) and gamma_ax w^{m+1} (tile and
// column halo); the in-plane taps then come from LDS and, in 3D, those of
// axis 0 from global memory (through the caches).  Neighbours beyond the
// padded array read 0.  The sums run in the same order as the point-wise
// definition: centre, then per axis the taps j = 1..R.
constexpr int kMadjRows = 8;

template <int R, int ND, bool Y2>
__global__ __launch_bounds__(256) void medium_adjoint_kernel(Dims d, StencilCoef cf, SpongeCoef sp,
                                                             MediumAdjParams mp)
{
    constexpr int ay = ND - 2, ax = ND - 1;
    constexpr int TW = kTileX + 2 * R, TH = kMadjRows + 2 * R;
    __shared__ float Yt[TH][TW];
    __shared__ float Zy[TH][kTileX];
    __shared__ float Zx[kMadjRows][TW];
    const int tid = (int)threadIdx.x;
    const int x0 = (int)blockIdx.x * kTileX, y0 = (int)blockIdx.y * kMadjRows;
    const int z = ND == 3 ? (int)blockIdx.z : 0;
    const int ny = d.n[ay], nx = d.n[ax];
    const long long base = ND == 3 ? (long long)z * d.st[0] : 0;
    const long long sty = d.st[ay];
    auto yv = [&](long long q) {
        if constexpr (Y2)
            return fmaf(mp.att[q], mp.w1[q] - mp.w2[q], mp.w1[q]);
        else
            return mp.w1[q];
    };
    for (int e = tid; e < TH * TW; e += 256) {
        const int ly = e / TW, lx = e - ly * TW;
        const int gy = y0 + ly - R, gx = x0 + lx - R;
        float v = 0.f;
        if (gy >= 0 && gy < ny && gx >= 0 && gx < nx)
            v = yv(base + gy * sty + gx);
        Yt[ly][lx] = v;
    }
    for (int e = tid; e < TH * kTileX; e += 256) {
        const int ly = e / kTileX, lx = e - ly * kTileX;
        const int gy = y0 + ly - R, gx = x0 + lx;
        float v = 0.f;
        if (gy >= 0 && gy < ny && gx < nx) {
            const long long q = base + gy * sty + gx;
            v = mp.gam[ay][q] * mp.w1[q];
        }
        Zy[ly][lx] = v;
    }
    for (int e = tid; e < kMadjRows * TW; e += 256) {
        const int ly = e / TW, lx = e - ly * TW;
        const int gy = y0 + ly, gx = x0 + lx - R;
        float v = 0.f;
        if (gy < ny && gx >= 0 && gx < nx) {
            const long long q = base + gy * sty + gx;
            v = mp.gam[ax][q] * mp.w1[q];
        }
        Zx[ly][lx] = v;
    }
    __syncthreads();
    const int lx = tid & 63;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int ly = (tid >> 6) * 2 + r;
        const int gy = y0 + ly, gx = x0 + lx;
        if (gy >= ny || gx >= nx)
            continue;
        int c[3];
        if constexpr (ND == 3) {
            c[0] = z;
            c[1] = gy;
            c[2] = gx;
        } else {
            c[0] = gy;
            c[1] = gx;
            c[2] = 0;
        }
        const long long p = base + gy * sty + gx;
        const float w1 = mp.w1[p];
        float lap_y = cf.c0 * Yt[ly + R][lx + R];
        float dens = 0.f;
#pragma unroll
        for (int a = 0; a < ND; ++a) {
            float sy = 0.f, sz = 0.f;
#pragma unroll
            for (int jj = 1; jj <= R; ++jj) {
                float yp, ym, zp, zm;
                if (a == ay) {
                    yp = Yt[ly + R + jj][lx + R];
                    ym = Yt[ly + R - jj][lx + R];
                    zp = Zy[ly + R + jj][lx];
                    zm = Zy[ly + R - jj][lx];
                } else if (a == ax) {
                    yp = Yt[ly + R][lx + R + jj];
                    ym = Yt[ly + R][lx + R - jj];
                    zp = Zx[ly][lx + R + jj];
                    zm = Zx[ly][lx + R - jj];
                } else {
                    // axis 0 of a 3D grid: the neighbouring planes
                    const long long st = d.st[0];
                    const bool in_p = c[0] + jj < d.n[0], in_m = c[0] - jj >= 0;
                    const long long qp = p + jj * st, qm = p - jj * st;
                    yp = in_p ? yv(qp) : 0.f;
                    ym = in_m ? yv(qm) : 0.f;
                    zp = in_p ? mp.gam[0][qp] * mp.w1[qp] : 0.f;
                    zm = in_m ? mp.gam[0][qm] * mp.w1[qm] : 0.f;
                }
                sy = fmaf(cf.c[a][jj], yp + ym, sy);
                sz = fmaf(cf.d[a][jj], zp - zm, sz);
            }
            lap_y += sy;
            dens += sz;
        }
        float eta = sponge_eta(d, sp, c);
        if (mp.att && mp.att_power == 0)
            eta += mp.att[p];
        mp.w0[p] = leapfrog(w1, mp.w2[p], mp.k[p], lap_y - dens, eta, sp.half_dt);
        if (mp.H)
            mp.G[p] = fmaf(w1, mp.H[p], mp.G[p]);
    }
}

// 3D form of the kernel above with one row per thread (512 threads, the same
// 64 x 8 tile): the axis-0 taps of a thread's point are loaded first, into
// registers, so that their loads are in flight together with the tile loads
// instead of starting after the block's barrier.
template <int R, bool Y2>
__global__ __launch_bounds__(512) void medium_adjoint_kernel3(Dims d, StencilCoef cf, SpongeCoef sp,
                                                              MediumAdjParams mp)
{
    constexpr int TW = kTileX + 2 * R, TH = kMadjRows + 2 * R;
    __shared__ float Yt[TH][TW];
    __shared__ float Zy[TH][kTileX];
    __shared__ float Zx[kMadjRows][TW];
    const int tid = (int)threadIdx.x;
    const int x0 = (int)blockIdx.x * kTileX, y0 = (int)blockIdx.y * kMadjRows;
    const int z = (int)blockIdx.z;
    const int n0 = d.n[0], ny = d.n[1], nx = d.n[2];
    const long long st0 = d.st[0], sty = d.st[1];
    const long long base = (long long)z * st0;
    const int lx = tid & 63, ly = tid >> 6;
    const int gy = y0 + ly, gx = x0 + lx;
    const bool inside = gy < ny && gx < nx;
    const long long p = base + gy * sty + gx;
    // axis-0 taps: raw values (the operand is formed after the barrier)
    float w1p[R], w1m[R], gp[R], gm[R], w2p[R], w2m[R], ap[R], am[R];
#pragma unroll
    for (int jj = 1; jj <= R; ++jj) {
        const bool in_p = inside && z + jj < n0, in_m = inside && z - jj >= 0;
        const long long qp = p + jj * st0, qm = p - jj * st0;
        w1p[jj - 1] = in_p ? mp.w1[qp] : 0.f;
        w1m[jj - 1] = in_m ? mp.w1[qm] : 0.f;
        gp[jj - 1] = in_p ? mp.gam[0][qp] : 0.f;
        gm[jj - 1] = in_m ? mp.gam[0][qm] : 0.f;
        if constexpr (Y2) {
            w2p[jj - 1] = in_p ? mp.w2[qp] : 0.f;
            w2m[jj - 1] = in_m ? mp.w2[qm] : 0.f;
            ap[jj - 1] = in_p ? mp.att[qp] : 0.f;
            am[jj - 1] = in_m ? mp.att[qm] : 0.f;
        }
    }
    auto yv = [&](long long q) {
        if constexpr (Y2)
            return fmaf(mp.att[q], mp.w1[q] - mp.w2[q], mp.w1[q]);
        else
            return mp.w1[q];
    };
    for (int e = tid; e < TH * TW; e += 512) {
        const int ty = e / TW, tx = e - ty * TW;
        const int yy = y0 + ty - R, xx = x0 + tx - R;
        float v = 0.f;
        if (yy >= 0 && yy < ny && xx >= 0 && xx < nx)
            v = yv(base + yy * sty + xx);
        Yt[ty][tx] = v;
    }
    for (int e = tid; e < TH * kTileX; e += 512) {
        const int ty = e / kTileX, tx = e - ty * kTileX;
        const int yy = y0 + ty - R, xx = x0 + tx;
        float v = 0.f;
        if (yy >= 0 && yy < ny && xx < nx) {
            const long long q = base + yy * sty + xx;
            v = mp.gam[1][q] * mp.w1[q];
        }
        Zy[ty][tx] = v;
    }
    for (int e = tid; e < kMadjRows * TW; e += 512) {
        const int ty = e / TW, tx = e - ty * TW;
        const int yy = y0 + ty, xx = x0 + tx - R;
        float v = 0.f;
        if (yy < ny && xx >= 0 && xx < nx) {
            const long long q = base + yy * sty + xx;
            v = mp.gam[2][q] * mp.w1[q];
        }
        Zx[ty][tx] = v;
    }
    __syncthreads();
    if (!inside)
        return;
    const int c[3] = {z, gy, gx};
    const float w1 = mp.w1[p];
    float lap_y = cf.c0 * Yt[ly + R][lx + R];
    float dens = 0.f;
    {
        float sy = 0.f, sz = 0.f;
#pragma unroll
        for (int jj = 1; jj <= R; ++jj) {
            float yp = w1p[jj - 1], ym = w1m[jj - 1];
            if constexpr (Y2) {
                // a point outside the grid loaded 0 for w1, w2 and att: 0 here too
                yp = fmaf(ap[jj - 1], w1p[jj - 1] - w2p[jj - 1], w1p[jj - 1]);
                ym = fmaf(am[jj - 1], w1m[jj - 1] - w2m[jj - 1], w1m[jj - 1]);
            }
            const float zp = gp[jj - 1] * w1p[jj - 1], zm = gm[jj - 1] * w1m[jj - 1];
            sy = fmaf(cf.c[0][jj], yp + ym, sy);
            sz = fmaf(cf.d[0][jj], zp - zm, sz);
        }
        lap_y += sy;
        dens += sz;
    }
    {
        float sy = 0.f, sz = 0.f;
#pragma unroll
        for (int jj = 1; jj <= R; ++jj) {
            sy = fmaf(cf.c[1][jj], Yt[ly + R + jj][lx + R] + Yt[ly + R - jj][lx + R], sy);
            sz = fmaf(cf.d[1][jj], Zy[ly + R + jj][lx] - Zy[ly + R - jj][lx], sz);
        }
        lap_y += sy;
        dens += sz;
    }
    {
        float sy = 0.f, sz = 0.f;
#pragma unroll
        for (int jj = 1; jj <= R; ++jj) {
            sy = fmaf(cf.c[2][jj], Yt[ly + R][lx + R + jj] + Yt[ly + R][lx + R - jj], sy);
            sz = fmaf(cf.d[2][jj], Zx[ly][lx + R + jj] - Zx[ly][lx + R - jj], sz);
        }
        lap_y += sy;
        dens += sz;
    }
    float eta = sponge_eta(d, sp, c);
    if (mp.att && mp.att_power == 0)
        eta += mp.att[p];
    mp.w0[p] = leapfrog(w1, mp.w2[p], mp.k[p], lap_y - dens, eta, sp.half_dt);
    if (mp.H)
        mp.G[p] = fmaf(w1, mp.H[p], mp.G[p]);
}

template <int R, int ND>
void launch_medium_adjoint_t(const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                             const MediumAdjParams& mp, hipStream_t s)
{
    if constexpr (ND == 3) {
        const dim3 g((unsigned)((d.n[2] + kTileX - 1) / kTileX),
                     (unsigned)((d.n[1] + kMadjRows - 1) / kMadjRows), (unsigned)d.n[0]);
        if (mp.att && mp.att_power == 2)
            hipLaunchKernelGGL((medium_adjoint_kernel3<R, true>), g, dim3(512), 0, s, d, cf, sp, mp);
        else
            hipLaunchKernelGGL((medium_adjoint_kernel3<R, false>), g, dim3(512), 0, s, d, cf, sp, mp);
        return;
    }
    const dim3 g((unsigned)((d.n[ND - 1] + kTileX - 1) / kTileX),
                 (unsigned)((d.n[ND - 2] + kMadjRows - 1) / kMadjRows), ND == 3 ? (unsigned)d.n[0] : 1u);
    if (mp.att && mp.att_power == 2)
        hipLaunchKernelGGL((medium_adjoint_kernel<R, ND, true>), g, dim3(256), 0, s, d, cf, sp, mp);
    else
        hipLaunchKernelGGL((medium_adjoint_kernel<R, ND, false>), g, dim3(256), 0, s, d, cf, sp, mp);
}

void launch_medium_adjoint(const Dims& d, int R, const StencilCoef& cf, const SpongeCoef& sp,
                           const MediumAdjParams& mp, hipStream_t s)
{
    if (R == 4)
        d.nd == 3 ? launch_medium_adjoint_t<4, 3>(d, cf, sp, mp, s)
                  : launch_medium_adjoint_t<4, 2>(d, cf, sp, mp, s);
    else
        d.nd == 3 ? launch_medium_adjoint_t<5, 3>(d, cf, sp, mp, s)
                  : launch_medium_adjoint_t<5, 2>(d, cf, sp, mp, s);
}

// One block per step-kernel block of the table's launch shape; each thread
// takes the table's entries tid, tid + 256, ...; the first entry of a point
// sums the point's run in entry order (so every point is written by one
// thread, and always in the same order).
__global__ __launch_bounds__(256) void inject_table_kernel(Dims d, LaunchShape ls, InjTable T,
                                                           const float* sig, int stride, int step,
                                                           const float* k, const float* att,
                                                           int att_power, SpongeCoef sp, float* out)
{
    const int b = blockIdx.x;
    const int e0 = T.ptr[b], e1 = T.ptr[b + 1];
    const int zci = b / ls.tiles_xy;
    const int tile = b - zci * ls.tiles_xy;
    const int y0 = (tile / ls.tiles_x) * ls.ty;
    const int x0 = (tile % ls.tiles_x) * kTileX;
    const int plane = ls.ty * kTileX;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
        const TileEntry head = T.ent[e];
        if (head.run <= 0)
            continue;
        const float v = tile_point_signal(T.ent + e, head, sig, stride, step);
        const int pz = head.local / plane;
        const int rem = head.local - pz * plane;
        int c[3];
        if (d.nd == 3) {
            c[0] = zci * ls.zc + pz;
            c[1] = y0 + rem / kTileX;
            c[2] = x0 + rem % kTileX;
        } else {
            c[0] = y0 + rem / kTileX;
            c[1] = x0 + rem % kTileX;
            c[2] = 0;
        }
        const long long p = d.nd == 3 ? c[0] * d.st[0] + c[1] * d.st[1] + c[2] : c[0] * d.st[0] + c[1];
        float eta = sponge_eta(d, sp, c);
        if (att && att_power == 0)
            eta += att[p];
        const float a = eta == 0.f ? 1.f : __builtin_amdgcn_rcpf(fmaf(eta, sp.half_dt, 1.f));
        out[p] = fmaf(a * k[p], v, out[p]);
    }
}

void launch_inject_table(const Dims& d, const LaunchShape& ls, const InjTable& T, const float* sig,
                         int stride, int step, const float* k, const float* att, int att_power,
                         const SpongeCoef& sp, float* out, hipStream_t s)
{
    if (ls.tile_blocks <= 0)
        return;
    hipLaunchKernelGGL(inject_table_kernel, dim3(ls.tile_blocks), dim3(256), 0, s, d, ls, T, sig,
                       stride, step, k, att, att_power, sp, out);
}

void launch_vp_check(const float* vp, long long n, unsigned* flags, hipStream_t s)
{
    launch_fill(reinterpret_cast<float*>(flags), 2, 0.f, s);
    hipLaunchKernelGGL(vp_check_kernel, dim3(grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024),
                       dim3(256), 0, s, vp, n, flags);
}

void launch_prep_medium(const Dims& d, const Fd1& fd, const float* vp, const float* rho,
                        const float* alpha0, int att_power, double dt, float* const gam[3],
                        float* att, hipStream_t s)
{
    long long n = (long long)d.n[0] * d.n[1] * d.n[2];
    hipLaunchKernelGGL(prep_medium_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, d, fd, vp, rho,
                       alpha0, att_power, dt, gam[0], gam[1], d.nd == 3 ? gam[2] : gam[1], att);
}

void launch_medium_check(const float* vp, const float* rho, const float* alpha0, long long n,
                         int att_power, double dt, unsigned* flags, hipStream_t s)
{
    launch_fill(reinterpret_cast<float*>(flags + 2), 2, 0.f, s);
    hipLaunchKernelGGL(medium_check_kernel, dim3(grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024),
                       dim3(256), 0, s, vp, rho, alpha0, n, att_power, dt, flags);
}

void launch_time_filter3(float* rows, int count, int nt, hipStream_t s)
{
    if (count <= 0 || nt <= 0)
        return;
    hipLaunchKernelGGL(time_filter3_kernel, dim3(count), dim3(256), sizeof(float) * (size_t)nt, s, rows,
                       nt);
}

int lowpass_taps(double dt, double f_max)
{
    return (int)std::ceil(2.0 / (f_max * dt));
}

void launch_lowpass(const float* in, float* out, int count, int nt, double dt, double f_max,
                    hipStream_t s)
{
    const int K = lowpass_taps(dt, f_max);
    const size_t lds = sizeof(float) * (size_t)(2 * K + 1 + nt);
    hipLaunchKernelGGL(lowpass_kernel, dim3(count), dim3(256), lds, s, in, out, nt, f_max * dt, K);
}

void launch_descent(float* vp, const float* g, const float* mask, long long n, float step,
                    float vmin, float vmax, unsigned* work, hipStream_t s)
{
    launch_fill(reinterpret_cast<float*>(work), 1, 0.f, s);
    const int blocks = grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024;
    hipLaunchKernelGGL(grad_absmax_kernel, dim3(blocks), dim3(256), 0, s, g, mask, n, work);
    hipLaunchKernelGGL(descent_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, vp, g, mask, n, step,
                       vmin, vmax, work);
}

void launch_prep_k(const Dims& d, const float* vp, double dt, float* k, hipStream_t s)
{
    long long n = (long long)d.n[0] * d.n[1] * d.n[2];
    hipLaunchKernelGGL(prep_k_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, d, vp, dt, k);
}

void launch_residual_misfit(const float* traces, const float* observed, float* residual,
                            long long n, double* misfit, double* partial, hipStream_t s)
{
    hipLaunchKernelGGL(residual_partial_kernel, dim3(kMisfitParts), dim3(256), 0, s, traces,
                       observed, residual, n, partial);
    hipLaunchKernelGGL(misfit_final_kernel, dim3(1), dim3(256), 0, s, partial, kMisfitParts, misfit);
}

void launch_finalize_dvp(const Dims& d, const float* G, const float* kdiv, const float* vp,
                         float* dvp, float* tmp0, float* tmp1, hipStream_t s)
{
    // P^T one axis at a time, innermost first; the first pass reads the
    // pitched field, later passes dense intermediates, the last writes dvp.
    const int nd = d.nd;
    long long ext[3] = {d.n[0], d.n[1], d.n[2]};
    const float* in = G;
    float* tmp[2] = {tmp0, tmp1};
    for (int a = nd - 1; a >= 0; --a) {
        long long m0 = 1, m2 = 1;
        for (int q = 0; q < a; ++q)
            m0 *= ext[q];
        for (int q = a + 1; q < nd; ++q)
            m2 *= ext[q];
        const long long s_outer = a == nd - 1 ? d.st[nd - 2] : ext[a] * m2;
        const long long s_axis = a == nd - 1 ? 1 : m2;
        float* out = a == 0 ? dvp : tmp[a & 1];
        const long long cnt = m0 * d.phys[a] * m2;
        hipLaunchKernelGGL(pad_transpose_axis_kernel, dim3(grid_for(cnt, 256)), dim3(256), 0, s, in,
                           a == nd - 1 ? kdiv : nullptr, s_outer, s_axis, out, m0, d.phys[a], m2,
                           d.nb, a == 0 ? vp : nullptr);
        ext[a] = d.phys[a];
        in = out;
    }
}

}  // namespace stride
