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

// Implicit contraction is off: every fused multiply-add is written out as
// fmaf, so the arithmetic of a point does not depend on how the compiler
// schedules the surrounding code (any two kernels that evaluate the same
// expressions compute the same bits).
#pragma clang fp contract(off)

#include <cstdlib>
#include <type_traits>

namespace stride {

// Tile shapes the kernels use (the host sizes launch shapes with these).
// 3D defaults (fastest on 316^3): forward 4 rows x 8 waves, adjoint 2 rows x 4 waves.
void tile_shape(int nd, bool adjoint, int* ry, int* waves)
{
    if (nd == 2) {
        const char* er = getenv(adjoint ? "STRIDE_RY2D_ADJ" : "STRIDE_RY2D");
        const char* ew = getenv(adjoint ? "STRIDE_WAVES2D_ADJ" : "STRIDE_WAVES2D");
        int r = er && *er ? atoi(er) : 4;
        int w = ew && *ew ? atoi(ew) : 4;
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
    int r = er && *er ? atoi(er) : (adjoint ? 2 : 4);
    int w = ew && *ew ? atoi(ew) : (adjoint ? 4 : 8);
    if (w != 8)
        w = 4;
    if (r != 1 && r != 2)
        r = 4;
    if (w == 4 && r == 1)
        r = 2;
    *ry = r;
    *waves = w;
}

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

__device__ __forceinline__ float leapfrog(float ctr, float prev, float kk, float rhs, float eta,
                                          float half_dt)
{
    if (eta == 0.f)
        return fmaf(kk, rhs, fmaf(2.f, ctr, -prev));
    const float a = 1.f / fmaf(eta, half_dt, 1.f);
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
            p.C[po[j]] = medium_out(ctr, lap, fmaf(mgy[j], dy, mgx[j] * dx), inj, lapb, SB[0], kk[j],
                                    mat[j], p.att_power, eta, sp.half_dt);
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
    int rbo[RY], roff[RY];
    bool rin[RY];
    float ey[RY];
    const int dxd = layer_depth(gx, n2, d.nb);
    const float ex = sp.e[2] * (float)(dxd * dxd);
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = y0 + wy * RY + j;
        rin[j] = xin && gy < n1;
        roff[j] = gy * s1 + gx;
        rbo[j] = rin[j] ? roff[j] * 4 : -1;
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

            float* Cz = p.C + (long long)z * s0;
            float* Gz = ADJ && MODE != kAdjPlain ? p.G + (long long)z * s0 : nullptr;
            float* Vz = MODE == kStepV ? p.V + (long long)z * s0 : nullptr;
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
                    __builtin_nontemporal_store(medium_out(ctr, lap, dens, inj, lapb, prev, kk[j], mm[3][j],
                                                           p.att_power, eta, sp.half_dt),
                                                Cz + roff[j]);
                    continue;
                }
                const float out = step_out<ADJ, MODE>(ctr, lap, inj, uu[j], bb[j], kk[j], eta, sp.half_dt);
                __builtin_nontemporal_store(out, Cz + roff[j]);
                if constexpr (MODE == kStepV)
                    __builtin_nontemporal_store(lap, Vz + roff[j]);
                if constexpr (MODE == kImageV) {
                    __builtin_nontemporal_store(fmaf(ctr, vw[j], fmaf(bb[j], vw2[j], gg[j])), Gz + roff[j]);
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
                    __builtin_nontemporal_store(image_out<MODE>(ctr, uc0, lu, uu[j], kk[j], gg[j]),
                                                Gz + roff[j]);
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

template <int R, bool ADJ, int RY, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void step2d_batched(Dims d, StencilCoef cf, LaunchShape ls,
                                                             const SlotStep* table)
{
    const SlotStep st = table[blockIdx.y];
    if (!st.active)
        return;
    step2d_body<R, ADJ, RY, WAVES>(d, cf, st.sp, st.p, ls, blockIdx.x);
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

template <int R, bool ADJ, int RY, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void step3d_batched(Dims d, StencilCoef cf, LaunchShape ls,
                                                             const SlotStep* table)
{
    const SlotStep st = table[blockIdx.y];
    if (!st.active)
        return;
    step3d_body<R, ADJ, RY, WAVES>(d, cf, st.sp, st.p, ls, blockIdx.x);
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

// 2D tile shapes with compiled kernels (rows per thread, waves); tile_shape()
// returns one of these.
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

template <int R, bool ADJ, int MODE>
void launch_step_t(const Dims& d, const StencilCoef& cf, const SpongeCoef& sp,
                   const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    const int nt = 64 * ls.waves;
    int smp_blocks = (p.smp.count * sample_lanes(p.smp.ntap) + nt - 1) / nt;
    dim3 grid(ls.tile_blocks_pad + smp_blocks);
    if (d.nd == 2) {
#define STRIDE_LAUNCH2D(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step2d_kernel<R, ADJ, RY_, W_, MODE>), grid, dim3(64 * (W_)), 0, s, d, cf, sp, \
                       p, ls)
        STRIDE_DISPATCH2D(STRIDE_LAUNCH2D);
#undef STRIDE_LAUNCH2D
        return;
    }
#define STRIDE_LAUNCH3D(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step3d_kernel<R, ADJ, RY_, W_, MODE>), grid, dim3(64 * (W_)), 0, s, d, cf, sp, \
                       p, ls)
    if (ls.waves == 8) {
        if (ls.ry == 1)
            STRIDE_LAUNCH3D(1, 8);
        else if (ls.ry == 2)
            STRIDE_LAUNCH3D(2, 8);
        else
            STRIDE_LAUNCH3D(4, 8);
    } else {
        if (ls.ry == 2)
            STRIDE_LAUNCH3D(2, 4);
        else
            STRIDE_LAUNCH3D(4, 4);
    }
#undef STRIDE_LAUNCH3D
}

template <int R, bool ADJ>
void launch_batched_t(const Dims& d, const StencilCoef& cf, const LaunchShape& ls,
                      const SlotStep* table, int nslots, int max_sample_threads, hipStream_t s)
{
    const int nt = 64 * ls.waves;
    int smp_blocks = (max_sample_threads + nt - 1) / nt;
    dim3 grid(ls.tile_blocks_pad + smp_blocks, nslots);
    if (d.nd == 2) {
#define STRIDE_LAUNCH2DB(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step2d_batched<R, ADJ, RY_, W_>), grid, dim3(64 * (W_)), 0, s, d, cf, ls, table)
        STRIDE_DISPATCH2D(STRIDE_LAUNCH2DB);
#undef STRIDE_LAUNCH2DB
        return;
    }
#define STRIDE_LAUNCH3DB(RY_, W_)                                                                  \
    hipLaunchKernelGGL((step3d_batched<R, ADJ, RY_, W_>), grid, dim3(64 * (W_)), 0, s, d, cf, ls, table)
    if (ls.waves == 8) {
        if (ls.ry == 1)
            STRIDE_LAUNCH3DB(1, 8);
        else if (ls.ry == 2)
            STRIDE_LAUNCH3DB(2, 8);
        else
            STRIDE_LAUNCH3DB(4, 8);
    } else {
        if (ls.ry == 2)
            STRIDE_LAUNCH3DB(2, 4);
        else
            STRIDE_LAUNCH3DB(4, 4);
    }
#undef STRIDE_LAUNCH3DB
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

void launch_step_mode(const Dims& d, int R, bool adjoint, int mode, const StencilCoef& cf,
                      const SpongeCoef& sp, const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    if (adjoint && mode == kImageV)
        R == 4 ? launch_step_t<4, true, kImageV>(d, cf, sp, ls, p, s)
               : launch_step_t<5, true, kImageV>(d, cf, sp, ls, p, s);
    else if (adjoint && mode == kAdjPlain)
        R == 4 ? launch_step_t<4, true, kAdjPlain>(d, cf, sp, ls, p, s)
               : launch_step_t<5, true, kAdjPlain>(d, cf, sp, ls, p, s);
    else if (adjoint)   // the adjoint of the fourth-order step runs kCorrect
        R == 4 ? launch_step_t<4, true, kCorrect>(d, cf, sp, ls, p, s)
               : launch_step_t<5, true, kCorrect>(d, cf, sp, ls, p, s);
    else if (mode == kStepV)
        R == 4 ? launch_step_t<4, false, kStepV>(d, cf, sp, ls, p, s)
               : launch_step_t<5, false, kStepV>(d, cf, sp, ls, p, s);
    else if (mode == kMedium)
        R == 4 ? launch_step_t<4, false, kMedium>(d, cf, sp, ls, p, s)
               : launch_step_t<5, false, kMedium>(d, cf, sp, ls, p, s);
    else if (mode == kPrep)
        R == 4 ? launch_step_t<4, false, kPrep>(d, cf, sp, ls, p, s)
               : launch_step_t<5, false, kPrep>(d, cf, sp, ls, p, s);
    else
        R == 4 ? launch_step_t<4, false, kCorrect>(d, cf, sp, ls, p, s)
               : launch_step_t<5, false, kCorrect>(d, cf, sp, ls, p, s);
}

void launch_step(const Dims& d, int R, bool adjoint, const StencilCoef& cf, const SpongeCoef& sp,
                 const LaunchShape& ls, const StepParams& p, hipStream_t s)
{
    if (R == 4)
        adjoint ? launch_step_t<4, true, kStep>(d, cf, sp, ls, p, s) : launch_step_t<4, false, kStep>(d, cf, sp, ls, p, s);
    else
        adjoint ? launch_step_t<5, true, kStep>(d, cf, sp, ls, p, s) : launch_step_t<5, false, kStep>(d, cf, sp, ls, p, s);
}

void launch_step_batched(const Dims& d, int R, bool adjoint, const StencilCoef& cf,
                         const LaunchShape& ls, const SlotStep* table, int nslots, int max_samples,
                         hipStream_t s)
{
    if (R == 4)
        adjoint ? launch_batched_t<4, true>(d, cf, ls, table, nslots, max_samples, s)
                : launch_batched_t<4, false>(d, cf, ls, table, nslots, max_samples, s);
    else
        adjoint ? launch_batched_t<5, true>(d, cf, ls, table, nslots, max_samples, s)
                : launch_batched_t<5, false>(d, cf, ls, table, nslots, max_samples, s);
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
