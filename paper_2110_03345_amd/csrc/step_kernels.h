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
// This header holds the step kernels and their launch templates; the
// translation units step2d.hip, step3d_fwd.hip and step3d_adj.hip each
// instantiate one family, so that they compile in parallel.
#pragma once

#include "common.h"

// Implicit contraction is off: every fused multiply-add is written out as
// fmaf, so the arithmetic of a point does not depend on how the compiler
// schedules the surrounding code (any two kernels that evaluate the same
// expressions compute the same bits).
#pragma clang fp contract(off)

#include <type_traits>

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

// Calls fn(integral_constant<I>) for I = 0..N-1 while it returns true; every
// I is a compile-time constant in the body (used to index register queues).
template <int N, int I = 0, class Fn>
__device__ __forceinline__ void unrolled_while(Fn&& fn)
{
    if constexpr (I < N) {
        if (fn(std::integral_constant<int, I>{}))
            unrolled_while<N, I + 1>(fn);
    }
}

// Raw buffer access (CDNA): a descriptor over [base, base + bytes) returns 0
// for any byte offset at or beyond `bytes`, so loads of points outside the
// grid need no branch: their offset is set to 0xffffffff, and a plane outside
// the grid gets bytes = 0.  Third descriptor word of the gfx9 family.
constexpr int kBufWord3 = 0x00020000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, kBufWord3);
}

__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int byte_off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, 0, 0);
}

// Store with the non-temporal policy (results are read back only in a later
// launch): a 32-bit offset into a per-plane descriptor, no 64-bit address.
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, int byte_off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, byte_off, 0, 2);
}

// The builtin returns the raw 32 bits; reinterpret them (no numeric conversion).
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int byte_off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// Streamed operands (read once per step: u^{n-1}, k, G) are loaded with the
// non-temporal cache policy so they do not evict the stencil field's halo.
#ifndef STRIDE_STREAM_AUX
#define STRIDE_STREAM_AUX 2
#endif
__device__ __forceinline__ float bload_stream(__amdgpu_buffer_rsrc_t r, int byte_off)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, STRIDE_STREAM_AUX));
}

__device__ __forceinline__ int layer_depth(int i, int n, int nb)
{
    int hi = n - 1 - nb;
    return i < nb ? nb - i : (i > hi ? i - hi : 0);
}

__device__ __forceinline__ void sample_block(const SampleSet& smp, const float* field, int step,
                                             int sb)
{
    if (sample_lanes(smp.ntap) == 1) {
        const int r = sb * (int)blockDim.x + (int)threadIdx.x;
        if (r >= smp.count)
            return;
        float acc = 0.f;
        const long long base = (long long)r * smp.ntap;
        for (int t = 0; t < smp.ntap; ++t)
            acc = fmaf(smp.w[base + t], field[smp.idx[base + t]], acc);
        float* o = smp.out + (long long)r * smp.out_stride + step;
        *o = smp.accumulate ? fmaf(smp.scale, acc, *o) : smp.scale * acc;
        return;
    }
    // one wave per point: lane l sums taps l, l + 64, ...; then a butterfly
    // reduction over the wave (a fixed order, so results are reproducible)
    const int lane = (int)threadIdx.x & 63;
    const int r = sb * ((int)blockDim.x >> 6) + ((int)threadIdx.x >> 6);
    if (r >= smp.count)
        return;
    const long long base = (long long)r * smp.ntap;
    float acc = 0.f;
    for (int t = lane; t < smp.ntap; t += 64)
        acc = fmaf(smp.w[base + t], field[smp.idx[base + t]], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        acc += __shfl_xor(acc, off, 64);
    if (lane == 0) {
        float* o = smp.out + (long long)r * smp.out_stride + step;
        *o = smp.accumulate ? fmaf(smp.scale, acc, *o) : smp.scale * acc;
    }
}

constexpr float kTwelfth = 1.f / 12.f;

// Leapfrog update with the sponge's damping: a = 1 / (1 + eta dt/2) by the
// hardware reciprocal (within 1 ulp; an IEEE division would cost about ten
// instructions per point, and most waves of a 3D grid touch the sponge).
__device__ __forceinline__ float leapfrog(float ctr, float prev, float kk, float rhs, float eta,
                                          float half_dt)
{
    if (eta == 0.f)
        return fmaf(kk, rhs, fmaf(2.f, ctr, -prev));
    const float a = __builtin_amdgcn_rcpf(fmaf(eta, half_dt, 1.f));
    const float b = fmaf(-eta, half_dt, 1.f) * a;
    return fmaf(a, fmaf(kk, rhs, 2.f * ctr), -(b * prev));
}

// 2D Laplacian at S[0] of an LDS tile with row length LW_.
template <int R, int LW_>
__device__ __forceinline__ float lap2d(const float* S, const StencilCoef& cf)
{
    float ay = 0.f, ax = 0.f;
#pragma unroll
    for (int q = R; q >= 1; --q) {
        ay = fmaf(cf.c[0][q], S[q * LW_] + S[-q * LW_], ay);
        ax = fmaf(cf.c[1][q], S[q] + S[-q], ax);
    }
    return fmaf(cf.c0, S[0], ay + ax);
}

// ----------------------------------------------------------------------- 2D
//
// One block = one 64 x TY tile, TY = WAVES * RY rows (RY per thread).  The
// tile of A (and U) with its R-wide halo is staged in LDS row by row: wave w
// loads tile rows w, w + WAVES, ..., each lane one column and lanes 0..2R-1
// one halo column as well.  Every load of the step is issued up front: the
// point values of B, K (and G), the LDS tile, and the tile's injection
// entries with their signal samples (the entry range comes from a uniform
// table read), so a tile with injected points costs two dependent round trips
// and any other tile one.  Injected values reach their points through a small
// LDS array, used only by tiles that have entries.  The 2D field fits one
// buffer descriptor (at most 2 GiB): offsets of points outside the grid are
// set to 0xffffffff and read 0.

// Signal sample of row `id`: s[step], or with FILT (the fourth-order step's
// source) (s[step-1] + 10 s[step] + s[step+1]) / 12, zero outside the record.
template <bool FILT>
__device__ __forceinline__ float sig_at(const float* sig, int id, int stride, int step)
{
    const float* s = sig + (long long)id * stride;
    if constexpr (!FILT) {
        return s[step];
    } else {
        const float sm = step >= 1 ? s[step - 1] : 0.f;
        const float sp = step + 1 < stride ? s[step + 1] : 0.f;
        return fmaf(10.f, s[step], sm + sp) / 12.f;
    }
}

// Sum of the signals of the point whose first entry is `head` (entry order).
template <bool FILT = false>
__device__ __forceinline__ float tile_point_signal(const TileEntry* ent, TileEntry head,
                                                   const float* sig, int stride, int step)
{
    float v = head.w * sig_at<FILT>(sig, head.id, stride, step);
    for (int k = 1; k < head.run; ++k) {
        const TileEntry e = ent[k];
        v = fmaf(e.w, sig_at<FILT>(sig, e.id, stride, step), v);
    }
    return v;
}

// Output of a step launch at one point (see StepMode).  ctr and lap: centre
// and Laplacian of the stencil field A, with the injected value already added
// except in the adjoint correction, which takes it apart as inj and adds it
// as k inj (A = q = k L w^{m+1}, D = w^{m+1}):
//   w^m = a (2 w^{m+1} + q + (k/12) L q + k inj) - b w^{m+2}.
// uu: the point field D; bb, kk: B and k.
template <bool ADJ, int MODE>
constexpr bool kInjApart = (ADJ && MODE == kCorrect) || MODE == kMedium;

template <bool ADJ, int MODE>
__device__ __forceinline__ float step_out(float ctr, float lap, float inj, float uu, float bb,
                                          float kk, float eta, float half_dt)
{
    if constexpr (MODE == kStep || MODE == kStepV || MODE == kImageV || MODE == kAdjPlain) {
        return leapfrog(ctr, bb, kk, lap, eta, half_dt);
    } else if constexpr (MODE == kPrep) {
        return kk * lap;
    } else {
        float rhs = fmaf(kk * kTwelfth, lap, ctr);
        if constexpr (ADJ)
            rhs = fmaf(kk, inj, rhs);
        return leapfrog(uu, bb, 1.f, rhs, eta, half_dt);
    }
}

// Output of a medium step.  lap = L u, dens = sum_a gamma_a D_a u, inj the
// injected value, lapb = L u^{n-1}, prev = u^{n-1}; at is the attenuation
// field: added to the damping (att_power 0) or weighting L u - L u^{n-1} (2).
__device__ __forceinline__ float medium_out(float ctr, float lap, float dens, float inj,
                                            float lapb, float prev, float kk, float at,
                                            int att_power, float eta, float half_dt)
{
    float rhs = lap + dens + inj;
    if (att_power == 2)
        rhs = fmaf(at, lap - lapb, rhs);
    else
        eta += at;
    return leapfrog(ctr, prev, kk, rhs, eta, half_dt);
}

// Imaging factor of a medium step for the gradient with respect to vp,
// dJ/dvp = (2/vp) sum_n w^{n+1} h^n (stored by the forward when V is given):
//   y = 2:  h = v + (att/2) (L u - L u^{n-1})                (att = beta = 2 alpha0 vp / dt),
//   y = 0:  h = v + (att a dt/4) ((2 u^{n-1} - 2 u) / k - v)  (att = 2 alpha0 vp, a the
//           step's damping factor with the attenuation),
// v the step's right-hand side L u + sum_a gamma_a D_a u + S (+ beta (L u - L u^{n-1})).
__device__ __forceinline__ float medium_h(float ctr, float lap, float dens, float inj, float lapb,
                                          float prev, float kk, float at, int att_power, float eta,
                                          float half_dt)
{
    float v = lap + dens + inj;
    if (att_power == 2) {
        const float dl = lap - lapb;
        v = fmaf(at, dl, v);
        return fmaf(0.5f * at, dl, v);
    }
    const float a = __builtin_amdgcn_rcpf(fmaf(eta + at, half_dt, 1.f));
    const float du = 2.f * (prev - ctr) / kk;
    return fmaf(at * a * (0.5f * half_dt), du - v, v);
}

// Imaging accumulator update of an adjoint launch.  Second order:
// G += w^{m+1} (L u^m + S^m) with ctr = w^{m+1}, lu = L u^m + S^m.  Fourth
// order accumulates k G, the gradient with respect to k times k:
//   H += p (w + q/12) + (k/12) w L p,   p = k (L u^m + St^m), q = k L w,
// with ctr = q, pc = p, lu = L p and uu = w = w^{m+1}.
template <int MODE>
__device__ __forceinline__ float image_out(float ctr, float pc, float lu, float uu, float kk,
                                           float gg)
{
    if constexpr (MODE == kCorrect)
        return fmaf((kk * kTwelfth) * uu, lu, fmaf(pc, fmaf(ctr, kTwelfth, uu), gg));
    else
        return fmaf(ctr, lu, gg);
}

template <int R, bool ADJ, int RY, int WAVES, int MODE = kStep>
__device__ __forceinline__ void step2d_body(const Dims& d, const StencilCoef& cf,
                                            const SpongeCoef& sp, const StepParams& p,
                                            const LaunchShape& ls, const int b)
{
    constexpr int NT = 64 * WAVES;
    constexpr int TY = WAVES * RY;
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int RW = (LH + WAVES - 1) / WAVES;    // tile rows loaded per wave
    constexpr bool MED = MODE == kMedium;
    constexpr bool ONE = MODE == kImageV || MODE == kAdjPlain;      // adjoint with one stencil field
    constexpr int NF = (ADJ && !ONE) || MED ? 2 : 1;   // stencil fields A (and U, or B)
    __shared__ float sF[NF][LH * LW];
    __shared__ float sS[NF][TY * kTileX];           // injected signal per tile point

    if (b >= ls.tile_blocks_pad) {
        sample_block(p.smp, p.A, p.step, b - ls.tile_blocks_pad);
        return;
    }
    const int tile = xcd_logical(b, ls.tile_blocks_pad);
    if (tile >= ls.tile_blocks)
        return;
    const int tyi = tile / ls.tiles_x;
    const int y0 = tyi * TY;
    const int x0 = (tile - tyi * ls.tiles_x) * kTileX;
    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int wy = tid >> 6;
    const int n0 = d.n[0], n1 = d.n[1];
    const int s0 = (int)d.st[0];
    const int fbytes = (int)(d.total * 4);
    const int gx = x0 + lx;
    const bool xin = gx < n1;

    // entry ranges of the tile (uniform); the forward correction pass injects
    // nothing, the adjoint one its receivers, and it images without a source term
    constexpr bool INJ = MODE != kCorrect || ADJ;
    constexpr bool IMG = ADJ && MODE != kCorrect && !ONE;
    int eb0 = 0, ne0 = 0;
    if constexpr (INJ) {
        eb0 = p.inj.ptr[tile];
        ne0 = p.inj.ptr[tile + 1] - eb0;
    }
    int eb1 = 0, ne1 = 0;
    if constexpr (IMG) {
        eb1 = p.img.ptr[tile];
        ne1 = p.img.ptr[tile + 1] - eb1;
    }

    // tile rows with halo: byte offsets of the column and the halo column
    const int hcol = lx < R ? x0 - R + lx : x0 + kTileX - R + lx;
    const int hlds = lx < R ? lx : kTileX + lx;
    const bool hin = lx < 2 * R && hcol >= 0 && hcol < n1;
    int ro[RW], ho[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const int r = wy + i * WAVES;
        const int gy = y0 - R + r;
        const bool rok = r < LH && gy >= 0 && gy < n0;
        ro[i] = rok && xin ? (gy * s0 + gx) * 4 : -1;
        ho[i] = rok && hin ? (gy * s0 + hcol) * 4 : -1;
    }
    float va[NF][RW], vh[NF][RW];
    const float* F1 = ADJ ? p.U : p.B;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        const auto rf = plane_rsrc(f == 0 ? p.A : F1, fbytes);
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            va[f][i] = bload(rf, ro[i]);
            vh[f][i] = bload(rf, ho[i]);
        }
    }
    int po[RY];
    float bb[RY], kk[RY], gg[RY], uu[RY], mgy[RY], mgx[RY], mat[RY], vv[RY], v2[RY];
    {
        const auto rb = plane_rsrc(p.B, fbytes);
        const auto rk = plane_rsrc(p.K, fbytes);
        const auto ru = plane_rsrc(p.D, fbytes);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int gy = y0 + wy * RY + j;
            po[j] = xin && gy < n0 ? gy * s0 + gx : -1;
            const int bo = po[j] >= 0 ? po[j] * 4 : -1;
            if constexpr (MODE != kPrep && !MED)
                bb[j] = bload(rb, bo);
            kk[j] = bload(rk, bo);
            if constexpr (MODE == kCorrect)
                uu[j] = bload(ru, bo);
            if constexpr (MED) {
                mgy[j] = bload(plane_rsrc(p.gam[0], fbytes), bo);
                mgx[j] = bload(plane_rsrc(p.gam[1], fbytes), bo);
                mat[j] = bload(plane_rsrc(p.att, fbytes), bo);
            }
        }
        if constexpr (ADJ && MODE != kAdjPlain) {
            const auto rg = plane_rsrc(p.G, fbytes);
#pragma unroll
            for (int j = 0; j < RY; ++j)
                gg[j] = bload(rg, po[j] >= 0 ? po[j] * 4 : -1);
        }
        if constexpr (MODE == kImageV) {
            const auto rv = plane_rsrc(p.V, fbytes);
            const auto r2 = plane_rsrc(p.V2 ? p.V2 : p.V, p.V2 ? fbytes : 0);
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                vv[j] = bload(rv, po[j] >= 0 ? po[j] * 4 : -1);
                v2[j] = bload(r2, po[j] >= 0 ? po[j] * 4 : -1);
            }
        }
    }

    // one entry per thread (more only in tiles with over NT entries)
    int il0 = -1, il1 = -1;
    float iv0 = 0.f, iv1 = 0.f;
    if (tid < ne0) {
        const TileEntry e = p.inj.ent[eb0 + tid];
        if (e.run > 0) {
            il0 = e.local;
            iv0 = tile_point_signal<MODE == kPrep>(p.inj.ent + eb0 + tid, e, p.inj_sig,
                                                   p.inj_stride, p.step);
        }
    }
    if constexpr (IMG) {
        if (tid < ne1) {
            const TileEntry e = p.img.ent[eb1 + tid];
            if (e.run > 0) {
                il1 = e.local;
                iv1 = tile_point_signal(p.img.ent + eb1 + tid, e, p.img_sig, p.img_stride, p.step);
            }
        }
    }

#pragma unroll
    for (int f = 0; f < NF; ++f) {
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const int r = wy + i * WAVES;
            if (r < LH) {
                sF[f][r * LW + lx + R] = va[f][i];
                if (lx < 2 * R)
                    sF[f][r * LW + hlds] = vh[f][i];
            }
        }
    }
    const bool inj_any = ne0 > 0;
    const bool img_any = IMG && ne1 > 0;
    if (inj_any)
#pragma unroll
        for (int j = 0; j < RY; ++j)
            sS[0][(wy * RY + j) * kTileX + lx] = 0.f;
    if (img_any)
#pragma unroll
        for (int j = 0; j < RY; ++j)
            sS[NF - 1][(wy * RY + j) * kTileX + lx] = 0.f;
    __syncthreads();
    if (inj_any || img_any) {
        if (il0 >= 0)
            sS[0][il0] = iv0;
        for (int e = tid + NT; e < ne0; e += NT) {
            const TileEntry en = p.inj.ent[eb0 + e];
            if (en.run > 0)
                sS[0][en.local] = tile_point_signal<MODE == kPrep>(p.inj.ent + eb0 + e, en, p.inj_sig,
                                                                   p.inj_stride, p.step);
        }
        if constexpr (IMG) {
            if (il1 >= 0)
                sS[1][il1] = iv1;
            for (int e = tid + NT; e < ne1; e += NT) {
                const TileEntry en = p.img.ent[eb1 + e];
                if (en.run > 0)
                    sS[1][en.local] =
                        tile_point_signal(p.img.ent + eb1 + e, en, p.img_sig, p.img_stride, p.step);
            }
        }
        __syncthreads();
    }

    if (!xin)
        return;
    const int dxd = layer_depth(gx, n1, d.nb);
    const float ex = sp.e[1] * (float)(dxd * dxd);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        if (po[j] < 0)
            break;
        const int ly = wy * RY + j;
        const float* SA = &sF[0][(ly + R) * LW + lx + R];
        const float ctr = SA[0];
        float lap = lap2d<R, LW>(SA, cf);
        float inj = 0.f;
        if (inj_any) {
            if constexpr (kInjApart<ADJ, MODE>)
                inj = sS[0][ly * kTileX + lx];
            else
                lap += sS[0][ly * kTileX + lx];
        }
        const int dyd = layer_depth(y0 + ly, n0, d.nb);
        const float eta = fmaf(sp.e[0], (float)(dyd * dyd), ex);
        if constexpr (MED) {
            float dy = 0.f, dx = 0.f;
#pragma unroll
            for (int q = R; q >= 1; --q) {
                dy = fmaf(cf.d[0][q], SA[q * LW] - SA[-q * LW], dy);
                dx = fmaf(cf.d[1][q], SA[q] - SA[-q], dx);
            }
            const float* SB = &sF[1][(ly + R) * LW + lx + R];
            const float lapb = lap2d<R, LW>(SB, cf);
            const float dens = fmaf(mgy[j], dy, mgx[j] * dx);
            p.C[po[j]] = medium_out(ctr, lap, dens, inj, lapb, SB[0], kk[j], mat[j], p.att_power, eta,
                                    sp.half_dt);
            if (p.V)   // gradient forward: the imaging factor, read once by the adjoint
                __builtin_nontemporal_store(medium_h(ctr, lap, dens, inj, lapb, SB[0], kk[j], mat[j],
                                                     p.att_power, eta, sp.half_dt),
                                            p.V + po[j]);
            continue;
        }
        p.C[po[j]] = step_out<ADJ, MODE>(ctr, lap, inj, uu[j], bb[j], kk[j], eta, sp.half_dt);
        if constexpr (MODE == kStepV)   // read once, by the adjoint much later
            __builtin_nontemporal_store(lap, p.V + po[j]);
        if constexpr (MODE == kImageV) {
            // with V2 absent its loads read 0 (empty descriptor): fma(B, 0, G) = G
            p.G[po[j]] = fmaf(ctr, vv[j], fmaf(bb[j], v2[j], gg[j]));
        } else if constexpr (ADJ && MODE != kAdjPlain) {
            const float* SU = &sF[NF - 1][(ly + R) * LW + lx + R];
            float lu = lap2d<R, LW>(SU, cf);
            if (img_any)
                lu += sS[NF - 1][ly * kTileX + lx];
            p.G[po[j]] = image_out<MODE>(ctr, SU[0], lu, uu[j], kk[j], gg[j]);
        }
    }
}

// ----------------------------------------------------------------------- 3D
//
// One block = one 64 x TY column tile marching along axis 0 over a chunk of
// planes.  Each thread keeps the 2R+1 axis-0 neighbours of its RY points in a
// rotating register queue (the march is unrolled by 2R+1 so that the queue
// never shifts).  The plane tile with its halo goes to a double-buffered LDS
// slot, so one barrier per plane suffices.  The march is software-pipelined:
// while plane z is computed, the loads of plane z+1 (the queue's lead plane,
// the halo, and the streamed point values of B, K, G) are in flight.  All
// global accesses are raw buffer accesses with per-plane descriptors: offsets
// outside the grid read 0 and drop stores, so no access needs a branch.

template <int R, bool ADJ, int RY, int WAVES, int MODE = kStep>
__device__ __forceinline__ void step3d_body(const Dims& d, const StencilCoef& cf,
                                            const SpongeCoef& sp, const StepParams& p,
                                            const LaunchShape& ls, const int b)
{
    constexpr int NT = 64 * WAVES;
    constexpr int TY = WAVES * RY;
    constexpr int LW = kTileX + 2 * R;
    constexpr int LH = TY + 2 * R;
    constexpr int Q = 2 * R + 1;
    constexpr int NYH = 2 * R * kTileX;             // halo rows above/below
    constexpr int NXH = 2 * R * TY;                 // halo columns left/right
    constexpr int HY = (NYH + NT - 1) / NT;
    constexpr int HX = (NXH + NT - 1) / NT;
    constexpr bool MED = MODE == kMedium;
    constexpr bool ONE = MODE == kImageV || MODE == kAdjPlain;      // adjoint with one stencil field
    constexpr int NF = (ADJ && !ONE) || MED ? 2 : 1;   // stencil fields: A (and U, or B)
    constexpr int PLANE = LH * LW;
    constexpr int PL = TY * kTileX;                 // block-local points per plane
    __shared__ float sF[2][NF][PLANE];
    __shared__ float sS[2][NF][PL];                 // injected signal per plane point
    __shared__ int2 sE[NF][NT];                     // entry (local point, value) per thread

    if (b >= ls.tile_blocks_pad) {
        sample_block(p.smp, p.A, p.step, b - ls.tile_blocks_pad);
        return;
    }
    const int lb = xcd_logical(b, ls.tile_blocks_pad);
    if (lb >= ls.tile_blocks)
        return;
    const int zci = lb / ls.tiles_xy;
    const int tile = lb - zci * ls.tiles_xy;
    const int y0 = (tile / ls.tiles_x) * TY;
    const int x0 = (tile % ls.tiles_x) * kTileX;
    const int n0 = d.n[0], n1 = d.n[1], n2 = d.n[2];
    const int z0 = zci * ls.zc;
    const int z1 = min(z0 + ls.zc, n0);
    const long long s0 = d.st[0];
    const int s1 = (int)d.st[1];
    const int tid = threadIdx.x;
    const int lx = tid & 63;
    const int wy = tid >> 6;
    const int gx = x0 + lx;
    const bool xin = gx < n2;
    const float* F[2] = {p.A, ADJ ? p.U : (MED ? p.B : p.A)};

    // plane-independent geometry: byte offsets within a plane (-1 = outside)
    const int plane_bytes = (int)(s0 * 4);
    int rbo[RY];
    bool rin[RY];
    float ey[RY];
    const int dxd = layer_depth(gx, n2, d.nb);
    const float ex = sp.e[2] * (float)(dxd * dxd);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = y0 + wy * RY + j;
        rin[j] = xin && gy < n1;
        rbo[j] = rin[j] ? (gy * s1 + gx) * 4 : -1;
        const int dyd = layer_depth(gy, n1, d.nb);
        ey[j] = fmaf(sp.e[1], (float)(dyd * dyd), ex);
    }
    int hy_l[HY], hy_o[HY];
#pragma unroll
    for (int h = 0; h < HY; ++h) {
        const int i = tid + h * NT;
        hy_l[h] = -1;
        hy_o[h] = -1;
        if (i < NYH) {
            const int hr = i / kTileX;
            const int c = i - hr * kTileX;
            const int ly = hr < R ? hr - R : TY + hr - R;
            const int gy = y0 + ly;
            const int g = x0 + c;
            hy_l[h] = (ly + R) * LW + c + R;
            if (gy >= 0 && gy < n1 && g < n2)
                hy_o[h] = (gy * s1 + g) * 4;
        }
    }
    int hx_l[HX], hx_o[HX];
#pragma unroll
    for (int h = 0; h < HX; ++h) {
        const int i = tid + h * NT;
        hx_l[h] = -1;
        hx_o[h] = -1;
        if (i < NXH) {
            const int row = i / (2 * R);
            const int cc = i - row * (2 * R);
            const int lxx = cc < R ? cc - R : kTileX + cc - R;
            const int g = x0 + lxx;
            const int gy = y0 + row;
            hx_l[h] = (row + R) * LW + lxx + R;
            if (g >= 0 && g < n2 && gy < n1)
                hx_o[h] = (gy * s1 + g) * 4;
        }
    }
    auto rsrc = [&](const float* f, int z) {
        const bool in = z >= 0 && z < n0;
        return plane_rsrc(f + (long long)(in ? z : 0) * s0, in ? plane_bytes : 0);
    };

    // queue slot (i + t) % Q holds plane z0 + i + t - R at march iteration i
    float q[NF][RY][Q];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int t = 0; t < 2 * R; ++t) {
            const auto r = rsrc(F[f], z0 - R + t);
#pragma unroll
            for (int j = 0; j < RY; ++j)
                q[f][j][t] = bload(r, rbo[j]);
        }

    float pl[NF][RY], phy[NF][HY], phx[NF][HX];
    float pb[RY], pk[RY], pg[RY], pu[RY], pm[4][RY], pv[RY], pv2[RY];
    auto prefetch = [&](int z) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const auto rz = rsrc(F[f], z);
            const auto rl = rsrc(F[f], z + R);
#pragma unroll
            for (int j = 0; j < RY; ++j)
                pl[f][j] = bload(rl, rbo[j]);
#pragma unroll
            for (int h = 0; h < HY; ++h)
                phy[f][h] = bload(rz, hy_o[h]);
#pragma unroll
            for (int h = 0; h < HX; ++h)
                phx[f][h] = bload(rz, hx_o[h]);
        }
        const auto rb = rsrc(p.B, z);
        const auto rk = rsrc(p.K, z);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            if constexpr (MODE != kPrep && !MED)
                pb[j] = bload_stream(rb, rbo[j]);
            pk[j] = bload_stream(rk, rbo[j]);
        }
        if constexpr (MED) {
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const auto rm = rsrc(m < 3 ? p.gam[m] : p.att, z);
#pragma unroll
                for (int j = 0; j < RY; ++j)
                    pm[m][j] = bload_stream(rm, rbo[j]);
            }
        }
        if constexpr (MODE == kCorrect) {
            const auto ru = rsrc(p.D, z);
#pragma unroll
            for (int j = 0; j < RY; ++j)
                pu[j] = bload_stream(ru, rbo[j]);
        }
        if constexpr (ADJ && MODE != kAdjPlain) {
            const auto rg = rsrc(p.G, z);
#pragma unroll
            for (int j = 0; j < RY; ++j)
                pg[j] = bload_stream(rg, rbo[j]);
        }
        if constexpr (MODE == kImageV) {
            const auto rv = rsrc(p.V, z);
            // with V2 absent the descriptor is empty and its loads read 0
            const auto r2 = p.V2 ? rsrc(p.V2, z) : plane_rsrc(p.V, 0);
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                pv[j] = bload_stream(rv, rbo[j]);
                pv2[j] = bload_stream(r2, rbo[j]);
            }
        }
    };

    // Injection entries of the block (uniform range).  Thread t takes entry t,
    // sums the signal over the point's run and parks (local point, value) in
    // LDS; before the barrier of each plane it writes the value of its entry
    // of that plane to the LDS plane array, where the point's thread takes
    // (and clears) it after the barrier.  Blocks with more than NT entries
    // read the rest at every plane.
    constexpr bool INJ = MODE != kCorrect || ADJ;
    constexpr bool IMG = ADJ && MODE != kCorrect && !ONE;
    int eb0 = 0, ne0 = 0;
    if constexpr (INJ) {
        eb0 = p.inj.ptr[lb];
        ne0 = p.inj.ptr[lb + 1] - eb0;
    }
    int eb1 = 0, ne1 = 0;
    if constexpr (IMG) {
        eb1 = p.img.ptr[lb];
        ne1 = p.img.ptr[lb + 1] - eb1;
    }
    const bool inj_any = ne0 > 0;
    const bool img_any = IMG && ne1 > 0;
    prefetch(z0);
    if (inj_any || img_any) {
        int il0 = -1, il1 = -1;
        float iv0 = 0.f, iv1 = 0.f;
        if (tid < ne0) {
            const TileEntry e = p.inj.ent[eb0 + tid];
            if (e.run > 0) {
                il0 = e.local;
                iv0 = tile_point_signal<MODE == kPrep>(p.inj.ent + eb0 + tid, e, p.inj_sig,
                                                       p.inj_stride, p.step);
            }
        }
        if constexpr (IMG) {
            if (tid < ne1) {
                const TileEntry e = p.img.ent[eb1 + tid];
                if (e.run > 0) {
                    il1 = e.local;
                    iv1 = tile_point_signal(p.img.ent + eb1 + tid, e, p.img_sig, p.img_stride, p.step);
                }
            }
        }
#pragma unroll
        for (int bsel = 0; bsel < 2; ++bsel)
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int j = 0; j < RY; ++j)
                    sS[bsel][f][(wy * RY + j) * kTileX + lx] = 0.f;
        sE[0][tid] = make_int2(il0, __float_as_int(iv0));
        if constexpr (IMG)
            sE[1][tid] = make_int2(il1, __float_as_int(iv1));
        __syncthreads();
        if (il0 >= 0 && il0 < PL)
            sS[0][0][il0] = iv0;
        if constexpr (IMG)
            if (il1 >= 0 && il1 < PL)
                sS[0][1][il1] = iv1;
    }
    // Entries beyond the first NT of the block, written at their plane.  A
    // block's entries are sorted by point, so their planes never decrease.
    // The adjoint (receiver sets of up to 512 taps a point fill some blocks
    // with thousands of entries) keeps a cursor per thread over its entries
    // (tid + NT, tid + 2 NT, ...) and at plane pz takes them until the first
    // of a later plane: every entry is read once per chunk, plus one
    // look-ahead per plane.  The forward step, whose source entries rarely
    // overflow, scans them at every plane and keeps its registers.
    int oc0 = tid + NT, oc1 = tid + NT;
    auto overflow = [&](auto filt, const InjTable& T, int eb, int ne, int& oc, const float* sig,
                        int stride, int pz, float* dst) {
        if constexpr (ADJ) {
            for (; oc < ne; oc += NT) {
                const TileEntry en = T.ent[eb + oc];
                const int ez = en.local / PL;
                if (ez > pz)
                    break;
                if (en.run > 0 && ez == pz)
                    dst[en.local - pz * PL] = tile_point_signal<decltype(filt)::value>(
                        T.ent + eb + oc, en, sig, stride, p.step);
            }
        } else {
            for (int e = tid + NT; e < ne; e += NT) {
                const TileEntry en = T.ent[eb + e];
                if (en.run > 0 && en.local / PL == pz)
                    dst[en.local - pz * PL] = tile_point_signal<decltype(filt)::value>(
                        T.ent + eb + e, en, sig, stride, p.step);
            }
        }
    };

    int buf = 0;
    for (int zb = z0; zb < z1; zb += Q) {
        unrolled_while<Q>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            constexpr int slot_lead = (u + 2 * R) % Q;
            constexpr int slot_c = (u + R) % Q;
            const int z = zb + u;
            if (z >= z1)
                return false;
            float bb[RY], kk[RY], gg[RY], uu[RY], mm[4][RY], vw[RY], vw2[RY];
            float* S = &sF[buf][0][0];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                float* Sf = S + f * PLANE;
#pragma unroll
                for (int j = 0; j < RY; ++j) {
                    q[f][j][slot_lead] = pl[f][j];
                    Sf[(wy * RY + j + R) * LW + lx + R] = q[f][j][slot_c];
                }
#pragma unroll
                for (int h = 0; h < HY; ++h)
                    if (hy_l[h] >= 0)
                        Sf[hy_l[h]] = phy[f][h];
#pragma unroll
                for (int h = 0; h < HX; ++h)
                    if (hx_l[h] >= 0)
                        Sf[hx_l[h]] = phx[f][h];
            }
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                bb[j] = MODE != kPrep && !MED ? pb[j] : 0.f;
                kk[j] = pk[j];
                gg[j] = ADJ && MODE != kAdjPlain ? pg[j] : 0.f;
                uu[j] = MODE == kCorrect ? pu[j] : 0.f;
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    mm[m][j] = MED ? pm[m][j] : 0.f;
                vw[j] = MODE == kImageV ? pv[j] : 0.f;
                vw2[j] = MODE == kImageV ? pv2[j] : 0.f;
            }
            if (z + 1 < z1)
                prefetch(z + 1);
            const int pz = z - z0;
            if (pz > 0 && (inj_any || img_any)) {
                // parked entry sets: the injection, and the imaging source term
#pragma unroll
                for (int f = 0; f < (IMG ? 2 : 1); ++f) {
                    const int2 e = sE[f][tid];
                    if (e.x >= 0 && e.x / PL == pz)
                        sS[buf][f][e.x - pz * PL] = __int_as_float(e.y);
                }
            }
            if (ne0 > NT)
                overflow(std::integral_constant<bool, MODE == kPrep>{}, p.inj, eb0, ne0, oc0,
                         p.inj_sig, p.inj_stride, pz, &sS[buf][0][0]);
            if constexpr (IMG)
                if (ne1 > NT)
                    overflow(std::false_type{}, p.img, eb1, ne1, oc1, p.img_sig, p.img_stride, pz,
                             &sS[buf][NF - 1][0]);
            __syncthreads();

            const auto rC = rsrc(p.C, z);
            const auto rG = rsrc(ADJ && MODE != kAdjPlain ? p.G : p.C, z);
            const auto rV = rsrc((MODE == kStepV || MED) && p.V ? p.V : p.C, z);
            const int dzd = layer_depth(z, n0, d.nb);
            const float ez = sp.e[0] * (float)(dzd * dzd);
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                if (!rin[j])
                    continue;
                const int ly = wy * RY + j;
                const float* SA = S;
                const float ctr = q[0][j][slot_c];
                float az = 0.f, ay = 0.f, ax = 0.f;
#pragma unroll
                for (int qq = R; qq >= 1; --qq) {
                    az = fmaf(cf.c[0][qq], q[0][j][(u + R + qq) % Q] + q[0][j][(u + R - qq) % Q], az);
                    ay = fmaf(cf.c[1][qq], SA[(ly + R + qq) * LW + lx + R] + SA[(ly + R - qq) * LW + lx + R], ay);
                    ax = fmaf(cf.c[2][qq], SA[(ly + R) * LW + lx + R + qq] + SA[(ly + R) * LW + lx + R - qq], ax);
                }
                float lap = fmaf(cf.c0, ctr, az + ay + ax);
                float inj = 0.f;
                if (inj_any) {
                    if constexpr (kInjApart<ADJ, MODE>)
                        inj = sS[buf][0][ly * kTileX + lx];
                    else
                        lap += sS[buf][0][ly * kTileX + lx];
                    sS[buf][0][ly * kTileX + lx] = 0.f;
                }
                const float eta = ez + ey[j];
                if constexpr (MED) {
                    const float* SB = S + PLANE;
                    float dz = 0.f, dy = 0.f, dx = 0.f, bz = 0.f, by = 0.f, bx = 0.f;
#pragma unroll
                    for (int qq = R; qq >= 1; --qq) {
                        dz = fmaf(cf.d[0][qq], q[0][j][(u + R + qq) % Q] - q[0][j][(u + R - qq) % Q], dz);
                        dy = fmaf(cf.d[1][qq], SA[(ly + R + qq) * LW + lx + R] - SA[(ly + R - qq) * LW + lx + R], dy);
                        dx = fmaf(cf.d[2][qq], SA[(ly + R) * LW + lx + R + qq] - SA[(ly + R) * LW + lx + R - qq], dx);
                        bz = fmaf(cf.c[0][qq], q[1][j][(u + R + qq) % Q] + q[1][j][(u + R - qq) % Q], bz);
                        by = fmaf(cf.c[1][qq], SB[(ly + R + qq) * LW + lx + R] + SB[(ly + R - qq) * LW + lx + R], by);
                        bx = fmaf(cf.c[2][qq], SB[(ly + R) * LW + lx + R + qq] + SB[(ly + R) * LW + lx + R - qq], bx);
                    }
                    const float prev = q[1][j][slot_c];
                    const float lapb = fmaf(cf.c0, prev, bz + by + bx);
                    const float dens = fmaf(mm[0][j], dz, fmaf(mm[1][j], dy, mm[2][j] * dx));
                    bstore_nt(rC, rbo[j], medium_out(ctr, lap, dens, inj, lapb, prev, kk[j], mm[3][j],
                                                     p.att_power, eta, sp.half_dt));
                    if (p.V)   // gradient forward: the imaging factor
                        bstore_nt(rV, rbo[j], medium_h(ctr, lap, dens, inj, lapb, prev, kk[j], mm[3][j],
                                                       p.att_power, eta, sp.half_dt));
                    continue;
                }
                const float out = step_out<ADJ, MODE>(ctr, lap, inj, uu[j], bb[j], kk[j], eta, sp.half_dt);
                bstore_nt(rC, rbo[j], out);
                if constexpr (MODE == kStepV)
                    bstore_nt(rV, rbo[j], lap);
                if constexpr (MODE == kImageV) {
                    bstore_nt(rG, rbo[j], fmaf(ctr, vw[j], fmaf(bb[j], vw2[j], gg[j])));
                } else if constexpr (ADJ && MODE != kAdjPlain) {
                    const float* SU = S + (NF - 1) * PLANE;
                    const float uc0 = q[NF - 1][j][slot_c];
                    float uz = 0.f, uy = 0.f, ux = 0.f;
#pragma unroll
                    for (int qq = R; qq >= 1; --qq) {
                        uz = fmaf(cf.c[0][qq], q[NF - 1][j][(u + R + qq) % Q] + q[NF - 1][j][(u + R - qq) % Q], uz);
                        uy = fmaf(cf.c[1][qq], SU[(ly + R + qq) * LW + lx + R] + SU[(ly + R - qq) * LW + lx + R], uy);
                        ux = fmaf(cf.c[2][qq], SU[(ly + R) * LW + lx + R + qq] + SU[(ly + R) * LW + lx + R - qq], ux);
                    }
                    float lu = fmaf(cf.c0, uc0, uz + uy + ux);
                    if (img_any) {
                        lu += sS[buf][NF - 1][ly * kTileX + lx];
                        sS[buf][NF - 1][ly * kTileX + lx] = 0.f;
                    }
                    bstore_nt(rG, rbo[j], image_out<MODE>(ctr, uc0, lu, uu[j], kk[j], gg[j]));
                }
            }
            buf ^= 1;
            return true;
        });
    }
}

// ------------------------------------------------------------ kernel entry points
//
// Single shot: parameters by value.  Batched: blockIdx.y selects a slot whose
// parameters (and sponge, which depends on the slot's dt) are read from a
// device table; inactive slots exit at once.  Both run the same body, so a
// shot computes the same bits alone and in a batch.

template <int R, bool ADJ, int RY, int WAVES, int MODE = kStep>
__global__ __launch_bounds__(64 * WAVES) void step2d_kernel(Dims d, StencilCoef cf, SpongeCoef sp,
                                                            StepParams p, LaunchShape ls)
{
    step2d_body<R, ADJ, RY, WAVES, MODE>(d, cf, sp, p, ls, blockIdx.x);
}

template <int R, bool ADJ, int RY, int WAVES, int MODE>
__global__ __launch_bounds__(64 * WAVES) void step2d_batched(Dims d, StencilCoef cf, LaunchShape ls,
                                                             const SlotStep* table)
{
    const SlotStep st = table[blockIdx.y];
    if (!st.active)
        return;
    step2d_body<R, ADJ, RY, WAVES, MODE>(d, cf, st.sp, st.p, ls, blockIdx.x);
}

// Occupancy target of a single-shot 3D kernel: 4 waves per SIMD (at most 128
// VGPRs) where that costs no spills, else left to the compiler.  (The batched
// kernels hold their slot's parameters in registers as well; they are left to
// the compiler, which keeps them free of spills.)
template <bool ADJ, int RY, int WAVES, int MODE>
constexpr int min_waves_3d()
{
    return (MODE == kStep || MODE == kStepV || MODE == kImageV || MODE == kAdjPlain) &&
                   (RY <= 2 || (!ADJ && WAVES == 8))
               ? 4
               : 1;
}

template <int R, bool ADJ, int RY, int WAVES, int MODE = kStep>
__global__ __launch_bounds__(64 * WAVES)
__attribute__((amdgpu_waves_per_eu(min_waves_3d<ADJ, RY, WAVES, MODE>())))
void step3d_kernel(Dims d, StencilCoef cf, SpongeCoef sp, StepParams p, LaunchShape ls)
{
    step3d_body<R, ADJ, RY, WAVES, MODE>(d, cf, sp, p, ls, blockIdx.x);
}

template <int R, bool ADJ, int RY, int WAVES, int MODE>
__global__ __launch_bounds__(64 * WAVES) void step3d_batched(Dims d, StencilCoef cf, LaunchShape ls,
                                                             const SlotStep* table)
{
    const SlotStep st = table[blockIdx.y];
    if (!st.active)
        return;
    step3d_body<R, ADJ, RY, WAVES, MODE>(d, cf, st.sp, st.p, ls, blockIdx.x);
}

// Tile shapes with compiled kernels (rows per thread, waves); tile_shape()
// returns one of these.  Without STRIDE_TILE_SWEEP: the 2D shape and the three
// 3D shapes (forward, adjoint / two-field steps, and adjoint steps imaging
// from v) of common.h.
#ifdef STRIDE_TILE_SWEEP
#define STRIDE_DISPATCH2D(L)                                                                      \
    do {                                                                                          \
        if (ls.waves == 8)                                                                        \
            L(4, 8);                                                                              \
        else if (ls.ry == 2)                                                                      \
            L(2, 4);                                                                              \
        else if (ls.ry == 8)                                                                      \
            L(8, 4);                                                                              \
        else                                                                                      \
            L(4, 4);                                                                              \
    } while (0)
#define STRIDE_DISPATCH3D(L)                                                                      \
    do {                                                                                          \
        if (ls.waves == 8) {                                                                      \
            if (ls.ry == 1)                                                                       \
                L(1, 8);                                                                          \
            else if (ls.ry == 2)                                                                  \
                L(2, 8);                                                                          \
            else                                                                                  \
                L(4, 8);                                                                          \
        } else {                                                                                  \
            if (ls.ry == 2)                                                                       \
                L(2, 4);                                                                          \
            else                                                                                  \
                L(4, 4);                                                                          \
        }                                                                                         \
    } while (0)
#else
#define STRIDE_DISPATCH2D(L) L(kRy2d, kWaves2d)
#define STRIDE_DISPATCH3D(L)                                                                      \
    do {                                                                                          \
        if constexpr (!ADJ) {                                                                     \
            if (ls.ry == kRy3dFwd && ls.waves == kWaves3dFwd) {                                   \
                L(kRy3dFwd, kWaves3dFwd);                                                         \
                break;                                                                            \
            }                                                                                     \
        }                                                                                         \
        if constexpr (ADJ && (MODE == kImageV || MODE == kAdjPlain)) {                            \
            if (ls.ry == kRy3dAdjV && ls.waves == kWaves3dAdjV) {                                 \
                L(kRy3dAdjV, kWaves3dAdjV);                                                       \
                break;                                                                            \
            }                                                                                     \
        }                                                                                         \
        L(kRy3dAdj, kWaves3dAdj);                                                                 \
    } while (0)
#endif

// Launch of one step kernel family: the tile blocks, then the sample blocks.
template <int R, bool ADJ, int MODE>
void launch2d_t(const Dims& d, const StencilCoef& cf, const SpongeCoef& sp, const LaunchShape& ls,
                const StepParams& p, hipStream_t s)
{
    const int nt = 64 * ls.waves;
    int smp_blocks = (p.smp.count * sample_lanes(p.smp.ntap) + nt - 1) / nt;
    dim3 grid(ls.tile_blocks_pad + smp_blocks);
#define STRIDE_LAUNCH2D(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step2d_kernel<R, ADJ, RY_, W_, MODE>), grid, dim3(64 * (W_)), 0, s, d, cf, sp, \
                       p, ls)
    STRIDE_DISPATCH2D(STRIDE_LAUNCH2D);
#undef STRIDE_LAUNCH2D
}

template <int R, bool ADJ, int MODE>
void launch3d_t(const Dims& d, const StencilCoef& cf, const SpongeCoef& sp, const LaunchShape& ls,
                const StepParams& p, hipStream_t s)
{
    const int nt = 64 * ls.waves;
    int smp_blocks = (p.smp.count * sample_lanes(p.smp.ntap) + nt - 1) / nt;
    dim3 grid(ls.tile_blocks_pad + smp_blocks);
#define STRIDE_LAUNCH3D(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step3d_kernel<R, ADJ, RY_, W_, MODE>), grid, dim3(64 * (W_)), 0, s, d, cf, sp, \
                       p, ls)
    STRIDE_DISPATCH3D(STRIDE_LAUNCH3D);
#undef STRIDE_LAUNCH3D
}

template <int R, bool ADJ, int MODE>
void batched2d_t(const Dims& d, const StencilCoef& cf, const LaunchShape& ls, const SlotStep* table,
                 int nslots, int max_sample_threads, hipStream_t s)
{
    const int nt = 64 * ls.waves;
    int smp_blocks = (max_sample_threads + nt - 1) / nt;
    dim3 grid(ls.tile_blocks_pad + smp_blocks, nslots);
#define STRIDE_LAUNCH2DB(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step2d_batched<R, ADJ, RY_, W_, MODE>), grid, dim3(64 * (W_)), 0, s, d, cf, ls, \
                       table)
    STRIDE_DISPATCH2D(STRIDE_LAUNCH2DB);
#undef STRIDE_LAUNCH2DB
}

template <int R, bool ADJ, int MODE>
void batched3d_t(const Dims& d, const StencilCoef& cf, const LaunchShape& ls, const SlotStep* table,
                 int nslots, int max_sample_threads, hipStream_t s)
{
    const int nt = 64 * ls.waves;
    int smp_blocks = (max_sample_threads + nt - 1) / nt;
    dim3 grid(ls.tile_blocks_pad + smp_blocks, nslots);
#define STRIDE_LAUNCH3DB(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step3d_batched<R, ADJ, RY_, W_, MODE>), grid, dim3(64 * (W_)), 0, s, d, cf, ls, \
                       table)
    STRIDE_DISPATCH3D(STRIDE_LAUNCH3DB);
#undef STRIDE_LAUNCH3DB
}

// Runtime (R, mode) to template arguments for one family.  Forward modes:
// kStep, kPrep, kCorrect, kMedium, kStepV; adjoint modes: kStep, kCorrect,
// kImageV, kAdjPlain.
template <bool THREE_D, bool ADJ, int R>
void launch_mode_r(int mode, const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                   const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
#define STRIDE_MODE_CASE(M_)                                                                      \
    case M_:                                                                                      \
        if constexpr (THREE_D)                                                                    \
            launch3d_t<R, ADJ, M_>(d, cf, sp, ls, p, s);                                          \
        else                                                                                      \
            launch2d_t<R, ADJ, M_>(d, cf, sp, ls, p, s);                                          \
        return;
    if constexpr (ADJ) {
        switch (mode) {
            STRIDE_MODE_CASE(kStep)
            STRIDE_MODE_CASE(kCorrect)
            STRIDE_MODE_CASE(kImageV)
            STRIDE_MODE_CASE(kAdjPlain)
        default:
            return;
        }
    } else {
        switch (mode) {
            STRIDE_MODE_CASE(kStep)
            STRIDE_MODE_CASE(kPrep)
            STRIDE_MODE_CASE(kCorrect)
            STRIDE_MODE_CASE(kMedium)
            STRIDE_MODE_CASE(kStepV)
        default:
            return;
        }
    }
#undef STRIDE_MODE_CASE
}

// Runtime mode to template arguments for the batched launches of one
// family.  Forward modes: kStep, kStepV, kPrep, kCorrect; adjoint modes:
// kStep, kImageV, kAdjPlain, kCorrect.
template <bool THREE_D, bool ADJ, int R>
void batched_mode_r(int mode, const Dims& d, const StencilCoef& cf, const LaunchShape& ls,
                    const SlotStep* table, int nslots, int max_sample_threads, hipStream_t s)
{
#define STRIDE_BMODE_CASE(M_)                                                                     \
    case M_:                                                                                      \
        if constexpr (THREE_D)                                                                    \
            batched3d_t<R, ADJ, M_>(d, cf, ls, table, nslots, max_sample_threads, s);             \
        else                                                                                      \
            batched2d_t<R, ADJ, M_>(d, cf, ls, table, nslots, max_sample_threads, s);             \
        return;
    if constexpr (ADJ) {
        switch (mode) {
            STRIDE_BMODE_CASE(kStep)
            STRIDE_BMODE_CASE(kImageV)
            STRIDE_BMODE_CASE(kAdjPlain)
            STRIDE_BMODE_CASE(kCorrect)
        default:
            return;
        }
    } else {
        switch (mode) {
            STRIDE_BMODE_CASE(kStep)
            STRIDE_BMODE_CASE(kStepV)
            STRIDE_BMODE_CASE(kPrep)
            STRIDE_BMODE_CASE(kCorrect)
        default:
            return;
        }
    }
#undef STRIDE_BMODE_CASE
}

}  // namespace
}  // namespace stride
