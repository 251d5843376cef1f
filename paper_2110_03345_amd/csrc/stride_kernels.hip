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

#include "common.h"

namespace stride {

namespace {

constexpr int kXcds = 8;  // MI355X: workgroups go round-robin over 8 XCDs

// Hardware places block b on XCD b % 8.  Map blocks so that each XCD owns a
// contiguous range of logical tiles: neighbouring tiles then share halo rows
// through the same L2.
__device__ __forceinline__ int xcd_logical(int b, int nblk_pad)
{
    int per = nblk_pad / kXcds;
    return (b % kXcds) * per + b / kXcds;
}

__device__ __forceinline__ int layer_depth(int i, int n, int nb)
{
    int hi = n - 1 - nb;
    return i < nb ? nb - i : (i > hi ? i - hi : 0);
}

__device__ __forceinline__ float tile_signal(const TileTable& t, int b0, int b1, long long gi,
                                             const float* sig, int stride, int step)
{
    float s = 0.f;
    for (int e = b0; e < b1; ++e)
        if (t.pidx[e] == gi)
            s += t.w[e] * sig[(long long)t.id[e] * stride + step];
    return s;
}

__device__ __forceinline__ void sample_block(const SampleSet& smp, const float* field, int step,
                                             int sb)
{
    int r = sb * kThreads + (int)threadIdx.x;
    if (r >= smp.count)
        return;
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < kMaxTaps; ++t)
        acc += smp.w[r * kMaxTaps + t] * field[smp.idx[r * kMaxTaps + t]];
    smp.out[(long long)r * smp.out_stride + step] = acc;
}

__device__ __forceinline__ float leapfrog(float ctr, float prev, float kk, float rhs, float eta,
                                          float half_dt)
{
    if (eta == 0.f)
        return fmaf(kk, rhs, 2.f * ctr - prev);
    float h = eta * half_dt;
    float a = 1.f / (1.f + h);
    float b = (1.f - h) * a;
    return a * (2.f * ctr + kk * rhs) - b * prev;
}

// ----------------------------------------------------------------------- 2D

template <int R, bool ADJ>
__global__ __launch_bounds__(kThreads) void step2d_kernel(Dims d, StencilCoef cf, SpongeCoef sp,
                                                          StepParams p, LaunchShape ls)
{
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = kTileY + 2 * R;
    __shared__ float sA[LH][LW];
    __shared__ float sU[ADJ ? LH : 1][ADJ ? LW : 1];

    const int b = blockIdx.x;
    if (b >= ls.tile_blocks_pad) {
        sample_block(p.smp, p.A, p.step, b - ls.tile_blocks_pad);
        return;
    }
    const int tile = xcd_logical(b, ls.tile_blocks_pad);
    if (tile >= ls.tile_blocks)
        return;
    const int y0 = (tile / ls.tiles_x) * kTileY;
    const int x0 = (tile % ls.tiles_x) * kTileX;
    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int wy = tid >> 6;
    const int n0 = d.n[0], n1 = d.n[1];
    const long long s0 = d.st[0];

    for (int i = tid; i < LH * LW; i += kThreads) {
        int r = i / LW;
        int c = i - r * LW;
        int gy = y0 - R + r;
        int gx = x0 - R + c;
        bool in = gy >= 0 && gy < n0 && gx >= 0 && gx < n1;
        long long gi = (long long)gy * s0 + gx;
        sA[r][c] = in ? p.A[gi] : 0.f;
        if constexpr (ADJ)
            sU[r][c] = in ? p.U[gi] : 0.f;
    }
    __syncthreads();

    const int gx = x0 + lx;
    if (gx >= n1)
        return;
    const int ib = p.inj.tile_ptr[tile], ie = p.inj.tile_ptr[tile + 1];
    int mb = 0, me = 0;
    if constexpr (ADJ) {
        mb = p.img.tile_ptr[tile];
        me = p.img.tile_ptr[tile + 1];
    }
    const int dxd = layer_depth(gx, n1, d.nb);

#pragma unroll
    for (int j = 0; j < kRowsPerThread; ++j) {
        const int ly = wy * kRowsPerThread + j;
        const int gy = y0 + ly;
        if (gy >= n0)
            break;
        const long long gi = (long long)gy * s0 + gx;
        const float ctr = sA[ly + R][lx + R];
        float ly_sum = 0.f, lx_sum = 0.f;
#pragma unroll
        for (int q = R; q >= 1; --q) {
            ly_sum = fmaf(cf.c[0][q], sA[ly + R + q][lx + R] + sA[ly + R - q][lx + R], ly_sum);
            lx_sum = fmaf(cf.c[1][q], sA[ly + R][lx + R + q] + sA[ly + R][lx + R - q], lx_sum);
        }
        float lap = fmaf(cf.c0, ctr, ly_sum + lx_sum);
        if (ib < ie)
            lap += tile_signal(p.inj, ib, ie, gi, p.inj_sig, p.inj_stride, p.step);
        const int dyd = layer_depth(gy, n0, d.nb);
        const float eta = sp.e[0] * (float)(dyd * dyd) + sp.e[1] * (float)(dxd * dxd);
        const float prev = p.B[gi];
        const float kk = p.K[gi];
        p.C[gi] = leapfrog(ctr, prev, kk, lap, eta, sp.half_dt);
        if constexpr (ADJ) {
            const float uc = sU[ly + R][lx + R];
            float uy = 0.f, ux = 0.f;
#pragma unroll
            for (int q = R; q >= 1; --q) {
                uy = fmaf(cf.c[0][q], sU[ly + R + q][lx + R] + sU[ly + R - q][lx + R], uy);
                ux = fmaf(cf.c[1][q], sU[ly + R][lx + R + q] + sU[ly + R][lx + R - q], ux);
            }
            float lu = fmaf(cf.c0, uc, uy + ux);
            if (mb < me)
                lu += tile_signal(p.img, mb, me, gi, p.img_sig, p.img_stride, p.step);
            p.G[gi] = fmaf(ctr, lu, p.G[gi]);
        }
    }
}

// ----------------------------------------------------------------------- 3D

template <int R, bool ADJ>
__global__ __launch_bounds__(kThreads) void step3d_kernel(Dims d, StencilCoef cf, SpongeCoef sp,
                                                          StepParams p, LaunchShape ls)
{
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = kTileY + 2 * R;
    constexpr int Q = 2 * R + 1;
    constexpr int RY = kRowsPerThread;
    __shared__ float sA[LH][LW];
    __shared__ float sU[ADJ ? LH : 1][ADJ ? LW : 1];

    const int b = blockIdx.x;
    if (b >= ls.tile_blocks_pad) {
        sample_block(p.smp, p.A, p.step, b - ls.tile_blocks_pad);
        return;
    }
    const int lb = xcd_logical(b, ls.tile_blocks_pad);
    if (lb >= ls.tile_blocks)
        return;
    const int zci = lb / ls.tiles_xy;
    const int tile = lb - zci * ls.tiles_xy;
    const int y0 = (tile / ls.tiles_x) * kTileY;
    const int x0 = (tile % ls.tiles_x) * kTileX;
    const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
    const int z0 = zci * ls.zc;
    const int z1 = min(z0 + ls.zc, n0);
    const long long s0 = d.st[0], s1 = d.st[1];
    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int wy = tid >> 6;
    const int gx = x0 + lx;
    const bool xin = gx < n2;

    float qa[RY][Q];
    float qu[ADJ ? RY : 1][ADJ ? Q : 1];
    bool rin[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = y0 + wy * RY + j;
        rin[j] = xin && gy < n1;
        const long long base = (long long)gy * s1 + gx;
#pragma unroll
        for (int t = 0; t < 2 * R; ++t) {
            const int z = z0 - R + t;
            const bool ok = rin[j] && z >= 0 && z < n0;
            qa[j][t] = ok ? p.A[base + (long long)z * s0] : 0.f;
            if constexpr (ADJ)
                qu[j][t] = ok ? p.U[base + (long long)z * s0] : 0.f;
        }
    }

    const int ib = p.inj.tile_ptr[tile], ie = p.inj.tile_ptr[tile + 1];
    int mb = 0, me = 0;
    if constexpr (ADJ) {
        mb = p.img.tile_ptr[tile];
        me = p.img.tile_ptr[tile + 1];
    }
    const int dxd = layer_depth(gx, n2, d.nb);

    for (int z = z0; z < z1; ++z) {
        const long long zoff = (long long)z * s0;
        // lead plane z + R into the register queues
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int gy = y0 + wy * RY + j;
            const bool ok = rin[j] && z + R < n0;
            const long long gi = (long long)(z + R) * s0 + (long long)gy * s1 + gx;
            qa[j][2 * R] = ok ? p.A[gi] : 0.f;
            if constexpr (ADJ)
                qu[j][2 * R] = ok ? p.U[gi] : 0.f;
            sA[wy * RY + j + R][lx + R] = qa[j][R];
            if constexpr (ADJ)
                sU[wy * RY + j + R][lx + R] = qu[j][R];
        }
        // halo rows above and below the tile (R rows each, 64 wide)
        for (int i = tid; i < 2 * R * kTileX; i += kThreads) {
            const int hr = i / kTileX;
            const int c = i - hr * kTileX;
            const int ly = hr < R ? hr - R : kTileY + hr - R;
            const int gy = y0 + ly;
            const int g = x0 + c;
            const bool ok = gy >= 0 && gy < n1 && g < n2;
            const long long gi = zoff + (long long)gy * s1 + g;
            sA[ly + R][c + R] = ok ? p.A[gi] : 0.f;
            if constexpr (ADJ)
                sU[ly + R][c + R] = ok ? p.U[gi] : 0.f;
        }
        // halo columns left and right of the tile (R columns each, 16 high)
        for (int i = tid; i < 2 * R * kTileY; i += kThreads) {
            const int row = i / (2 * R);
            const int cc = i - row * (2 * R);
            const int lxx = cc < R ? cc - R : kTileX + cc - R;
            const int g = x0 + lxx;
            const int gy = y0 + row;
            const bool ok = g >= 0 && g < n2 && gy < n1;
            const long long gi = zoff + (long long)gy * s1 + g;
            sA[row + R][lxx + R] = ok ? p.A[gi] : 0.f;
            if constexpr (ADJ)
                sU[row + R][lxx + R] = ok ? p.U[gi] : 0.f;
        }
        __syncthreads();

        const int dzd = layer_depth(z, n0, d.nb);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            if (!rin[j])
                continue;
            const int ly = wy * RY + j;
            const int gy = y0 + ly;
            const long long gi = zoff + (long long)gy * s1 + gx;
            const float ctr = qa[j][R];
            float az = 0.f, ay = 0.f, ax = 0.f;
#pragma unroll
            for (int q = R; q >= 1; --q) {
                az = fmaf(cf.c[0][q], qa[j][R + q] + qa[j][R - q], az);
                ay = fmaf(cf.c[1][q], sA[ly + R + q][lx + R] + sA[ly + R - q][lx + R], ay);
                ax = fmaf(cf.c[2][q], sA[ly + R][lx + R + q] + sA[ly + R][lx + R - q], ax);
            }
            float lap = fmaf(cf.c0, ctr, az + ay + ax);
            if (ib < ie)
                lap += tile_signal(p.inj, ib, ie, gi, p.inj_sig, p.inj_stride, p.step);
            const int dyd = layer_depth(gy, n1, d.nb);
            const float eta = sp.e[0] * (float)(dzd * dzd) + sp.e[1] * (float)(dyd * dyd) +
                              sp.e[2] * (float)(dxd * dxd);
            const float prev = p.B[gi];
            const float kk = p.K[gi];
            p.C[gi] = leapfrog(ctr, prev, kk, lap, eta, sp.half_dt);
            if constexpr (ADJ) {
                const float uc = qu[j][R];
                float uz = 0.f, uy = 0.f, ux = 0.f;
#pragma unroll
                for (int q = R; q >= 1; --q) {
                    uz = fmaf(cf.c[0][q], qu[j][R + q] + qu[j][R - q], uz);
                    uy = fmaf(cf.c[1][q], sU[ly + R + q][lx + R] + sU[ly + R - q][lx + R], uy);
                    ux = fmaf(cf.c[2][q], sU[ly + R][lx + R + q] + sU[ly + R][lx + R - q], ux);
                }
                float lu = fmaf(cf.c0, uc, uz + uy + ux);
                if (mb < me)
                    lu += tile_signal(p.img, mb, me, gi, p.img_sig, p.img_stride, p.step);
                p.G[gi] = fmaf(ctr, lu, p.G[gi]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RY; ++j) {
#pragma unroll
            for (int t = 0; t < 2 * R; ++t) {
                qa[j][t] = qa[j][t + 1];
                if constexpr (ADJ)
                    qu[j][t] = qu[j][t + 1];
            }
        }
    }
}

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

// Residual and misfit J = 1/2 sum r^2 accumulated in FP64 by one block with a
// fixed reduction order (bitwise reproducible).
__global__ __launch_bounds__(1024) void residual_misfit_kernel(const float* traces,
                                                               const float* observed,
                                                               float* residual, long long n,
                                                               double* misfit)
{
    __shared__ double part[1024];
    double acc = 0.0;
    for (long long i = threadIdx.x; i < n; i += 1024) {
        float r = traces[i] - observed[i];
        residual[i] = r;
        acc += (double)r * (double)r;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *misfit = 0.5 * part[0];
}

// dvp = P^T (2 G / vp_pad): every physical cell collects the padded cells that
// replicate it (the strip behind an edge cell, the corner block behind a corner).
__global__ void finalize_dvp_kernel(Dims d, const float* G, const float* vp, float* dvp)
{
    long long nphys = (long long)d.phys[0] * d.phys[1] * d.phys[2];
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < nphys; i += stride) {
        int c[3];
        long long r = i;
        for (int a = 2; a >= 0; --a) {
            c[a] = (int)(r % d.phys[a]);
            r /= d.phys[a];
        }
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            if (a >= d.nd) {
                lo[a] = hi[a] = 0;
                continue;
            }
            lo[a] = c[a] == 0 ? 0 : c[a] + d.nb;
            hi[a] = c[a] == d.phys[a] - 1 ? c[a] + 2 * d.nb : c[a] + d.nb;
        }
        float acc = 0.f;
        for (int a0 = lo[0]; a0 <= hi[0]; ++a0)
            for (int a1 = lo[1]; a1 <= hi[1]; ++a1)
                for (int a2 = lo[2]; a2 <= hi[2]; ++a2) {
                    long long gi = (long long)a0 * d.st[0] + (long long)a1 * (d.nd > 1 ? d.st[1] : 0) +
                                   (d.nd > 2 ? a2 : 0);
                    acc += G[gi];
                }
        dvp[i] = 2.f * acc / vp[i];
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

template <int R, bool ADJ>
void launch_step_t(const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                   const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    int smp_blocks = (p.smp.count + kThreads - 1) / kThreads;
    dim3 grid(ls.tile_blocks_pad + smp_blocks);
    if (d.nd == 2)
        hipLaunchKernelGGL((step2d_kernel<R, ADJ>), grid, dim3(kThreads), 0, s, d, cf, sp, p, ls);
    else
        hipLaunchKernelGGL((step3d_kernel<R, ADJ>), grid, dim3(kThreads), 0, s, d, cf, sp, p, ls);
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

void launch_step(const Dims& d, int R, bool adjoint, const StencilCoef& cf, const SpongeCoef& sp,
                 const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    if (R == 4)
        adjoint ? launch_step_t<4, true>(d, cf, sp, ls, p, s) : launch_step_t<4, false>(d, cf, sp, ls, p, s);
    else
        adjoint ? launch_step_t<5, true>(d, cf, sp, ls, p, s) : launch_step_t<5, false>(d, cf, sp, ls, p, s);
}

void launch_sample(const SampleSet& smp, const float* field, int step, hipStream_t s)
{
    if (smp.count <= 0)
        return;
    int blocks = (smp.count + kThreads - 1) / kThreads;
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

void launch_vp_check(const float* vp, long long n, unsigned* flags, hipStream_t s)
{
    launch_fill(reinterpret_cast<float*>(flags), 2, 0.f, s);
    hipLaunchKernelGGL(vp_check_kernel, dim3(grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024),
                       dim3(256), 0, s, vp, n, flags);
}

void launch_prep_k(const Dims& d, const float* vp, double dt, float* k, hipStream_t s)
{
    long long n = (long long)d.n[0] * d.n[1] * d.n[2];
    hipLaunchKernelGGL(prep_k_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, d, vp, dt, k);
}

void launch_residual_misfit(const float* traces, const float* observed, float* residual,
                            long long n, double* misfit, hipStream_t s)
{
    hipLaunchKernelGGL(residual_misfit_kernel, dim3(1), dim3(1024), 0, s, traces, observed, residual,
                       n, misfit);
}

void launch_finalize_dvp(const Dims& d, const float* G, const float* vp, float* dvp, hipStream_t s)
{
    long long n = (long long)d.phys[0] * d.phys[1] * d.phys[2];
    hipLaunchKernelGGL(finalize_dvp_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, d, G, vp, dvp);
}

}  // namespace stride
