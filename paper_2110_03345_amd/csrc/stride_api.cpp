// Host side of the acoustic FWI library: plan construction (validation,
// bi/tri-linear taps, per-tile injection tables), workspace layout, the
// forward and adjoint time loops, binomial checkpointing over a pool of
// wavefields, and the exported C ABI (include/stride_hip.h).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "plan.h"

using namespace stride;

namespace {
thread_local std::string g_err;
}  // namespace

int stride::fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr) STRIDE_HIP_TRY(expr)

namespace {

long long round_up(long long v, long long a) { return (v + a - 1) / a * a; }

#ifdef STRIDE_TILE_SWEEP
int env_int(const char* name, int dflt)
{
    const char* s = getenv(name);
    return s && *s ? atoi(s) : dflt;
}
#endif

// Central second-derivative weights of the (2r+1)-point stencil, as exact
// rationals (unique solution of the Taylor moment conditions).
bool fd_weights(int order, double* c)
{
    if (order == 8) {
        const double w[] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
        std::memcpy(c, w, sizeof(w));
        return true;
    }
    if (order == 10) {
        const double w[] = {-5269.0 / 1800.0, 5.0 / 3.0, -5.0 / 21.0, 5.0 / 126.0, -5.0 / 1008.0,
                            1.0 / 3150.0};
        std::memcpy(c, w, sizeof(w));
        return true;
    }
    return false;
}

// Centred first-derivative weights d_1..d_r of the (2r+1)-point antisymmetric
// stencil (exact rationals of the Taylor moment conditions).
bool fd1_weights(int order, double* dw)
{
    if (order == 8) {
        const double w[] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
        std::memcpy(dw, w, sizeof(w));
        return true;
    }
    if (order == 10) {
        const double w[] = {0.0, 5.0 / 6.0, -5.0 / 21.0, 5.0 / 84.0, -5.0 / 504.0, 1.0 / 1260.0};
        std::memcpy(dw, w, sizeof(w));
        return true;
    }
    return false;
}

LaunchShape make_shape(const Dims& d, int zc, int ry, int waves)
{
    LaunchShape ls{};
    int nx = d.n[d.nd - 1], ny = d.n[d.nd - 2];
    const int ty = ry * waves;
    ls.ty = ty;
    ls.ry = ry;
    ls.waves = waves;
    ls.tiles_x = (nx + kTileX - 1) / kTileX;
    ls.tiles_y = (ny + ty - 1) / ty;
    ls.tiles_xy = ls.tiles_x * ls.tiles_y;
    if (d.nd == 3) {
        ls.zc = std::max(1, std::min(zc, d.n[0]));
        ls.nzc = (d.n[0] + ls.zc - 1) / ls.zc;
    } else {
        ls.zc = 1;
        ls.nzc = 1;
    }
    ls.tile_blocks = ls.tiles_xy * ls.nzc;
    ls.tile_blocks_pad = (int)round_up(ls.tile_blocks, 8);
    return ls;
}

// Planes per 3D block.  Short chunks give many independent blocks (the march
// is latency-bound, so parallelism wins over the 2R lead-in planes each chunk
// re-reads, which mostly hit L2).  On 316^3: 32 for the 64 x 32 forward tile,
// 16 for the 64 x 8 adjoint tile.  (STRIDE_TILE_SWEEP builds read STRIDE_ZC.)
int default_zc(const Dims& d, bool adjoint)
{
    if (d.nd != 3)
        return 1;
#ifdef STRIDE_TILE_SWEEP
    int want = env_int("STRIDE_ZC", 0);
    if (want > 0)
        return want;
#endif
    return adjoint ? kZc3dAdj : kZc3dFwd;
}

int pitch_align()
{
#ifdef STRIDE_TILE_SWEEP
    return std::max(1, env_int("STRIDE_PITCH_ALIGN", kPitchAlign));
#else
    return kPitchAlign;
#endif
}

// Taps of a set of points: T per point, flat.
struct TapSet {
    int T = 0;
    std::vector<long long> idx;   // flat padded index
    std::vector<double> w;
    std::vector<int> coord;       // padded coordinates, 3 per tap
};

// Zeroth-order modified Bessel function of the first kind (power series).
double bessel_i0(double z)
{
    double term = 1.0, sum = 1.0;
    const double q = 0.25 * z * z;
    for (int k = 1; k < 200 && term > 1e-17 * sum; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
    }
    return sum;
}

// Kaiser-windowed sinc (Hicks 2002) at a node offset x cells from the point:
// sinc(x) I0(b sqrt(1 - (x/r)^2)) / I0(b), r = kSincHalfWidth, b = 6.31.
double windowed_sinc(double x)
{
    const double r = kSincHalfWidth, b = 6.31, pi = 3.14159265358979323846;
    if (std::fabs(x) > r)
        return 0.0;
    const double sc = x == 0.0 ? 1.0 : std::sin(pi * x) / (pi * x);
    const double q = x / r;
    return sc * bessel_i0(b * std::sqrt(1.0 - q * q)) / bessel_i0(b);
}

int taps_per_point(int nd, int interp)
{
    const int m = interp == 1 ? 2 * kSincHalfWidth : 2;
    return nd == 3 ? m * m * m : m * m;
}

// Taps of physical coordinates (metres from physical node 0): bi/tri-linear
// (2 nodes per axis) or windowed sinc (2 r nodes per axis, weights the
// product of the per-axis weights; a point on a node gets that node alone).
int make_taps(const stride_plan& P, const double* xyz, int count, TapSet& out, const char* what)
{
    const bool sinc = P.g.interp == 1;
    const int m = sinc ? 2 * kSincHalfWidth : 2;
    out.T = taps_per_point(P.nd, P.g.interp);
    out.idx.assign((size_t)count * out.T, 0);
    out.w.assign((size_t)count * out.T, 0.0);
    out.coord.assign((size_t)count * out.T * 3, 0);
    for (int p = 0; p < count; ++p) {
        int first[3] = {0, 0, 0};
        double w1[3][2 * kSincHalfWidth] = {};
        for (int a = 0; a < P.nd; ++a) {
            double x = xyz[(size_t)p * P.nd + a];
            double dx = P.g.spacing[a];
            double xmax = (double)(P.g.shape[a] - 1) * dx;
            double tol = 1e-9 * dx;
            if (!(x >= -tol && x <= xmax + tol))
                return fail(STRIDE_E_GEOMETRY,
                            "%s %d: coordinate %g on axis %d is outside the physical grid [0, %g]",
                            what, p, x, a, xmax);
            double gx = x / dx + (double)P.nb;
            long long i = (long long)std::floor(gx);
            i = std::min<long long>(std::max<long long>(i, 0), P.dims.n[a] - 2);
            double f = gx - (double)i;
            if (std::fabs(f) < 1e-9)
                f = 0.0;
            if (std::fabs(1.0 - f) < 1e-9)
                f = 1.0;
            if (!sinc) {
                first[a] = (int)i;
                w1[a][0] = 1.0 - f;
                w1[a][1] = f;
                continue;
            }
            if (f == 1.0) {
                i += 1;
                f = 0.0;
            }
            first[a] = (int)i - kSincHalfWidth + 1;
            if (first[a] < 0 || first[a] + m - 1 > P.dims.n[a] - 1)
                return fail(STRIDE_E_GEOMETRY,
                            "%s %d: the windowed-sinc taps on axis %d reach beyond the padded "
                            "grid (needs %d cells from its edge; sponge_cells is %d)",
                            what, p, a, kSincHalfWidth, P.nb);
            for (int j = 0; j < m; ++j) {
                const long long node = first[a] + j;
                w1[a][j] = f == 0.0 ? (node == i ? 1.0 : 0.0)
                                    : windowed_sinc((double)node - ((double)i + f));
            }
        }
        for (int t = 0; t < out.T; ++t) {
            long long lin = 0;
            double w = 1.0;
            int rem = t;
            const size_t k = (size_t)p * out.T + t;
            for (int a = 0; a < P.nd; ++a) {
                const int j = rem % m;
                rem /= m;
                const int c = first[a] + j;
                out.coord[k * 3 + a] = c;
                lin += (long long)c * P.dims.st[a];
                w *= w1[a][j];
            }
            out.idx[k] = lin;
            out.w[k] = w;
        }
    }
    return STRIDE_OK;
}

struct HostTiles {
    std::vector<int> ptr;
    std::vector<TileEntry> ent;
};

// Injection entries of every tap with a nonzero weight, grouped by block of a
// launch shape (2D: tile; 3D: tile and chunk of zc planes, block index
// chunk * tiles_xy + tile), sorted by block-local point and in (point, tap)
// order within a point.
HostTiles build_tiles(const stride_plan& P, const TapSet& taps, double scale,
                      const LaunchShape& ls)
{
    HostTiles T;
    const int plane = ls.ty * kTileX;   // block-local points per plane
    const size_t npts = taps.T ? taps.w.size() / taps.T : 0;
    std::vector<std::vector<TileEntry>> per(ls.tile_blocks);
    for (size_t p = 0; p < npts; ++p)
        for (int t = 0; t < taps.T; ++t) {
            const size_t k = p * taps.T + t;
            if (taps.w[k] == 0.0)
                continue;
            const int* c = &taps.coord[k * 3];
            const int cy = c[P.nd - 2], cx = c[P.nd - 1];
            const int ty = cy / ls.ty, tx = cx / kTileX;
            int zci = 0, pz = 0;
            if (P.nd == 3) {
                zci = c[0] / ls.zc;
                pz = c[0] - zci * ls.zc;
            }
            const int local = pz * plane + (cy - ty * ls.ty) * kTileX + (cx - tx * kTileX);
            const size_t blk = (size_t)zci * ls.tiles_xy + (size_t)ty * ls.tiles_x + tx;
            per[blk].push_back(TileEntry{local, 0, (int)p, (float)(taps.w[k] * scale)});
        }
    T.ptr.assign(ls.tile_blocks + 1, 0);
    for (int t = 0; t < ls.tile_blocks; ++t) {
        auto& v = per[t];
        std::stable_sort(v.begin(), v.end(),
                         [](const TileEntry& a, const TileEntry& b) { return a.local < b.local; });
        for (size_t i = 0; i < v.size();) {
            size_t j = i;
            while (j < v.size() && v[j].local == v[i].local)
                ++j;
            v[i].run = (int)(j - i);
            i = j;
        }
        T.ptr[t + 1] = T.ptr[t] + (int)v.size();
        T.ent.insert(T.ent.end(), v.begin(), v.end());
    }
    return T;
}

void flatten_sample(const TapSet& taps, double scale, std::vector<long long>& idx,
                    std::vector<float>& w)
{
    idx = taps.idx;
    w.resize(taps.w.size());
    for (size_t k = 0; k < taps.w.size(); ++k)
        w[k] = (float)(taps.w[k] * scale);
}

int validate_grid(const stride_grid_t* g)
{
    if (!g)
        return fail(STRIDE_E_INVALID_ARG, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3)
        return fail(STRIDE_E_INVALID_ARG, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->space_order != 8 && g->space_order != 10)
        return fail(STRIDE_E_INVALID_ARG, "space_order must be 8 or 10 (got %d)", g->space_order);
    if (g->sponge_cells < 0)
        return fail(STRIDE_E_INVALID_ARG, "sponge_cells must be >= 0");
    if (g->nt < 2)
        return fail(STRIDE_E_INVALID_ARG, "nt must be >= 2 (got %d)", g->nt);
    if (g->time_order != 0 && g->time_order != 2 && g->time_order != 4)
        return fail(STRIDE_E_INVALID_ARG, "time_order must be 2 or 4 (got %d)", g->time_order);
    if (g->interp != 0 && g->interp != 1)
        return fail(STRIDE_E_INVALID_ARG, "interp must be 0 (linear) or 1 (windowed sinc), got %d",
                    g->interp);
    if (g->checkpointing != 0 && g->checkpointing != 1)
        return fail(STRIDE_E_INVALID_ARG,
                    "checkpointing must be 0 (library's choice) or 1 (binomial), got %d",
                    g->checkpointing);
    if (g->boundary != 0 && g->boundary != 1)
        return fail(STRIDE_E_INVALID_ARG, "boundary must be 0 (sponge) or 1 (PML), got %d",
                    g->boundary);
    if (g->boundary == 1 && g->time_order == 4)
        return fail(STRIDE_E_INVALID_ARG, "the PML is offered with second-order time only");
    if (!(g->dt > 0) || !std::isfinite(g->dt))
        return fail(STRIDE_E_INVALID_ARG, "dt must be positive");
    if (!(g->sponge_vref >= 0) || !std::isfinite(g->sponge_vref))
        return fail(STRIDE_E_INVALID_ARG, "sponge_vref must be >= 0");
    long long total = 1;
    for (int a = 0; a < g->ndim; ++a) {
        if (g->shape[a] < 2)
            return fail(STRIDE_E_INVALID_ARG, "shape[%d] must be >= 2", a);
        if (!(g->spacing[a] > 0) || !std::isfinite(g->spacing[a]))
            return fail(STRIDE_E_INVALID_ARG, "spacing[%d] must be positive", a);
        long long np = g->shape[a] + 2LL * g->sponge_cells;
        if (np > (1 << 30))
            return fail(STRIDE_E_INVALID_ARG, "padded axis %d too large", a);
        total *= np;
    }
    if (total > (1LL << 40))
        return fail(STRIDE_E_INVALID_ARG, "grid too large");
    return STRIDE_OK;
}

}  // namespace

// ------------------------------------------------------------ workspace

Layout stride::layout_of(const stride_plan& P)
{
    Layout L;
    L.field = (size_t)round_up(P.dims.total * 4, 256);
    L.scratch = 256 + kMisfitParts * sizeof(double);   // flags | misfit partial sums
    L.traces = (size_t)round_up((long long)P.nrec * P.nt * 4, 256);
    // k, u, u (, p) (, two psi_a and one chi_a per axis with the PML)
    L.fixed_fwd = L.scratch + ((P.torder == 4 ? 4 : 3) + (P.boundary == 1 ? 3 * P.nd : 0)) * L.field;
    // k, G, w, w, traces, residual (, p and q of the fourth-order adjoint)
    L.fixed_grad = L.scratch + (P.torder == 4 ? 6 : 4) * L.field + 2 * L.traces;
    L.medium = L.scratch + (size_t)(4 + P.nd + 1) * L.field;
    // the medium gradient keeps every step's imaging factor: G and nt - 1 fields more;
    // checkpointed, G, h^m and a discarded u^{m+1} plus the state pool
    L.grad_medium = L.medium + (size_t)P.nt * L.field + 2 * L.traces;
    L.grad_medium_fixed = L.medium + 3 * L.field + 2 * L.traces;
    return L;
}

int stride::grad_ws(const stride_plan& P, void* ws, size_t bytes, GradWs& W)
{
    if (P.boundary == 1)
        return fail(STRIDE_E_INVALID_ARG, "the PML is offered for forward solves only");
    Layout L = layout_of(P);
    if (!ws)
        return fail(STRIDE_E_INVALID_ARG, "workspace is NULL");
    if ((uintptr_t)ws % 256)
        return fail(STRIDE_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (bytes < L.fixed_grad + 4 * L.field)
        return fail(STRIDE_E_WORKSPACE, "gradient workspace needs at least %zu bytes (got %zu)",
                    L.fixed_grad + 4 * L.field, bytes);
    long long nfields = (long long)((bytes - L.fixed_grad) / L.field);
    int s = snaps_for_fields(P.nt, nfields);
    if (s < 0)
        return fail(STRIDE_E_WORKSPACE, "workspace too small for checkpointing");
    ScheduleStats st = cached_schedule(P.nt, s)->stats;
    char* b = (char*)ws;
    W.flags = (unsigned*)b;
    W.partial = (double*)(b + 256);
    b += L.scratch;
    W.k = (float*)b;
    b += L.field;
    W.G = (float*)b;
    b += L.field;
    W.w[0] = (float*)b;
    b += L.field;
    W.w[1] = (float*)b;
    b += L.field;
    W.traces = (float*)b;
    b += L.traces;
    W.residual = (float*)b;
    b += L.traces;
    W.p = W.q = nullptr;
    if (P.torder == 4) {
        W.p = (float*)b;
        b += L.field;
        W.q = (float*)b;
        b += L.field;
    }
    // every field the workspace holds: the binomial schedule uses the first
    // peak_fields, the segmented-history path all of them
    W.pool.clear();
    for (long long f = 0; f < nfields; ++f) {
        W.pool.push_back((float*)b);
        b += L.field;
    }
    W.peak = st.peak_fields;
    W.snaps = s;
    return STRIDE_OK;
}

int stride::fwd_ws(const stride_plan& P, void* ws, size_t bytes, FwdWs& F)
{
    Layout L = layout_of(P);
    if (!ws || (uintptr_t)ws % 256)
        return fail(STRIDE_E_INVALID_ARG, "workspace must be a 256-byte aligned device pointer");
    if (bytes < L.fixed_fwd)
        return fail(STRIDE_E_WORKSPACE, "forward workspace needs %zu bytes (got %zu)", L.fixed_fwd,
                    bytes);
    char* b = (char*)ws;
    F.flags = (unsigned*)b;
    F.k = (float*)(b + L.scratch);
    F.u[0] = (float*)(b + L.scratch + L.field);
    F.u[1] = (float*)(b + L.scratch + 2 * L.field);
    F.p = P.torder == 4 ? (float*)(b + L.scratch + 3 * L.field) : nullptr;
    for (int a = 0; a < 3; ++a)
        F.psi[0][a] = F.psi[1][a] = F.chi[a] = nullptr;
    if (P.boundary == 1) {
        char* q = b + L.scratch + 3 * L.field;
        for (int a = 0; a < P.nd; ++a) {
            F.psi[0][a] = (float*)q;
            F.psi[1][a] = (float*)(q + L.field);
            F.chi[a] = (float*)(q + 2 * L.field);
            q += 3 * L.field;
        }
    }
    return STRIDE_OK;
}

int stride::check_cfl(const stride_plan& P, double vmax)
{
    double inv2 = 0;
    for (int a = 0; a < P.nd; ++a)
        inv2 += 1.0 / (P.g.spacing[a] * P.g.spacing[a]);
    // leapfrog: theta = dt^2 v^2 lambda sum 1/dx^2 <= 4; with the fourth-order
    // correction the update factor is 2 - theta + theta^2/12, stable for theta <= 12
    double courant = P.g.dt * vmax * std::sqrt(P.nyquist * inv2);
    const double limit = P.torder == 4 ? 2.0 * std::sqrt(3.0) : 2.0;
    if (!(courant <= limit))
        return fail(STRIDE_E_CFL,
                    "dt %g with vp_max %g violates the stability limit of the order-%d scheme "
                    "(dt vp sqrt(lambda sum 1/dx^2) = %.4f > %.4f)",
                    P.g.dt, vmax, P.torder, courant, limit);
    return STRIDE_OK;
}

int stride::check_vp(const stride_plan& P, const float* vp, unsigned* flags, hipStream_t s)
{
    long long n = 1;
    for (int a = 0; a < P.nd; ++a)
        n *= P.g.shape[a];
    launch_vp_check(vp, n, flags, s);
    unsigned host[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(host, flags, sizeof(host), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (host[1])
        return fail(STRIDE_E_INVALID_ARG, "vp contains non-positive or non-finite values");
    float vmax;
    std::memcpy(&vmax, &host[0], sizeof(float));
    return check_cfl(P, vmax);
}

StepParams stride::base_params(const stride_plan& P)
{
    StepParams p{};
    p.inj = P.src_inj;
    p.inj_stride = P.nt;
    p.img = P.src_img;
    p.img_stride = P.nt;
    return p;
}

// Segments of the segmented history for nt steps in a pool of `fields`
// fields: the smallest count K whose buffer (the longest segment) and K - 2
// stored start states plus a working pair fit, which leaves the fewest steps
// before the last segment.  Segment ends are even.  False when none fits.
bool stride::make_segments(long long nt, long long fields, std::vector<int>& starts, int& vbuf)
{
    for (long long K = 2;; ++K) {
        const long long S = fields - 2 * (K - 1);   // buffer beside K - 1 field pairs
        const long long Se = S & ~1LL;
        if (Se < 2)
            return false;
        long long last = std::max(0LL, nt - S);
        last += last & 1;
        if ((K - 1) * Se < last)
            continue;
        long long q = (last + K - 2) / (K - 1);
        q += q & 1;
        starts.clear();
        for (long long j = 0; j < last; j += q)
            starts.push_back((int)j);
        starts.push_back((int)last);
        const long long buf = std::max(nt - last, q);
        if (buf + 2 * ((long long)starts.size() - 1) > fields)
            return false;
        vbuf = (int)buf;
        return true;
    }
}

// Full history when every state fits; otherwise the segmented history when a
// cost model of the step kernels prefers it to the binomial schedule (whose
// adjoint recomputes L u^m itself).  Step costs relative to the plain
// second-order forward step, measured on MI355X (3D 316^3 / 2D 1104^2):
// second order, forward keeping v 1.18 / 1.04, adjoint imaging from v in
// pairs 1.48 / 1.30, fused adjoint 2.04 / 1.69; fourth order, forward 2.0
// (two launches, keeping p or not), adjoint from the kept p 3.13 / 2.63
// (two launches), binomial adjoint 3.98 / 3.53 (three).  The segment count is
// the smallest whose buffer and stored start states fit, which leaves the
// fewest steps to recompute.
GradPath stride::grad_path(const stride_plan& P, long long fields, int snaps)
{
    GradPath g;
    const long long nt = P.nt;
    const long long fb = cached_schedule(P.nt, snaps)->stats.forward_steps;
    g.forward_steps = fb * (P.torder == 4 ? 2 : 1);
    if (fb <= nt - 1 && fields >= nt) {
        g.kind = GradPath::kFull;
        return g;
    }
    if (P.g.checkpointing == 1)
        return g;
    const bool d3 = P.nd == 3;
    // per forward step (f: plain, fv: keeping v or p) and adjoint step (a:
    // imaging from the kept v or p, fused: the binomial path's own)
    double c_f = 1.0, c_fv = d3 ? 1.18 : 1.04, c_a = d3 ? 1.48 : 1.30, c_fused = d3 ? 2.04 : 1.69;
    if (P.torder == 4) {
        // two launches per forward step either way; the adjoint keeps its
        // correction and q launches and drops the p launch
        c_f = c_fv = 2.0;
        c_a = d3 ? 3.13 : 2.63;
        c_fused = d3 ? 3.98 : 3.53;
    }
    const double cost_b = c_f * (double)fb + c_fused * (double)nt;
    std::vector<int> st;
    int vbuf = 0;
    if (!make_segments(nt, fields, st, vbuf))
        return g;
    const long long last = st.back();
    const double cost_s = c_f * (double)last + c_fv * (double)(nt - 1) + c_a * (double)nt;
    if (cost_s < cost_b) {
        g.kind = GradPath::kSegmented;
        g.starts = std::move(st);
        g.vbuf = vbuf;
        g.forward_steps = (nt - 1 + last) * (P.torder == 4 ? 2 : 1);
    }
    return g;
}

// ------------------------------------------------------------ step cursor

StepCursor::StepCursor(int nt, int snaps, int pool_fields, bool in_place)
    : cs_(cached_schedule(nt, snaps)), in_place_(in_place)
{
    ref_.assign(pool_fields, 0);
    for (int f = pool_fields - 1; f >= 2; --f)
        freelist_.push_back(f);
    ref_[0] = ref_[1] = 1;
}

int StepCursor::alloc()
{
    if (freelist_.empty()) {
        overflow_ = true;
        return -1;
    }
    int f = freelist_.back();
    freelist_.pop_back();
    ref_[f] = 1;
    return f;
}

void StepCursor::release(int f)
{
    if (--ref_[f] == 0)
        freelist_.push_back(f);
}

void StepCursor::unget(const StepOp& op)
{
    back_ = op;
    have_back_ = true;
}

bool StepCursor::next(StepOp& op)
{
    if (have_back_) {
        have_back_ = false;
        op = back_;
        return true;
    }
    const std::vector<Action>& sched = cs_->actions;
    while (!overflow_) {
        if (target_ >= 0 && idx_ < target_) {
            // one forward step of the current Advance
            int old_prev = prev_;
            int out = in_place_ && ref_[prev_] == 1 ? prev_ : alloc();
            if (out < 0)
                return false;
            op = StepOp{false, idx_, cur_, old_prev, out, !reversed_};
            if (out != old_prev)
                release(old_prev);
            prev_ = cur_;
            cur_ = out;
            ++idx_;
            if (idx_ >= target_) {
                target_ = -1;
                ++pc_;
            }
            return true;
        }
        if (pc_ >= sched.size())
            return false;
        const Action& a = sched[pc_];
        switch (a.type) {
        case Act::Advance:
            if (idx_ < a.step) {
                target_ = a.step;
                continue;
            }
            ++pc_;
            continue;
        case Act::Store:
            snaps_[a.step] = {cur_, prev_};
            ++ref_[cur_];
            ++ref_[prev_];
            ++pc_;
            continue;
        case Act::Free: {
            auto it = snaps_.find(a.step);
            release(it->second.first);
            release(it->second.second);
            snaps_.erase(it);
            ++pc_;
            continue;
        }
        case Act::Restore: {
            auto it = snaps_.find(a.step);
            release(cur_);
            release(prev_);
            cur_ = it->second.first;
            prev_ = it->second.second;
            ++ref_[cur_];
            ++ref_[prev_];
            idx_ = a.step;
            ++pc_;
            continue;
        }
        case Act::Reverse:
            op = StepOp{true, a.step, cur_, prev_, -1, false};
            reversed_ = true;
            ++pc_;
            return true;
        }
    }
    return false;
}

namespace {

// ------------------------------------------------------------ phase timing

// Tracing of the time loops: when enabled on a thread, every solve records a
// HIP event pair around its forward time loop and its adjoint time loop on the
// solve's stream and counts the step launches in between.
struct PhaseTimer {
    bool on = false;
    struct Rec {
        hipEvent_t a, b;
        int kind;   // 0 forward loop, 1 adjoint loop, 2 recomputation inside 1
        long long steps, launches;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;

    hipEvent_t ev()
    {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        return e;
    }
    int begin(hipStream_t s)
    {
        if (!on)
            return -1;
        Rec r{ev(), ev(), 0, 0, 0};
        if (!r.a || !r.b)
            return -1;
        (void)hipEventRecord(r.a, s);
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void end(int id, hipStream_t s, int kind, long long steps, long long launches)
    {
        if (id < 0)
            return;
        recs[id].kind = kind;
        recs[id].steps = steps;
        recs[id].launches = launches;
        (void)hipEventRecord(recs[id].b, s);
    }
};

thread_local PhaseTimer g_timer;

// ------------------------------------------------------------ output checks

// Non-finite outputs (STRIDE_E_NONFINITE): while enabled on the calling thread
// (the default), a solve entry point scans what it wrote, each array into one
// bit of a flag word in the workspace's scratch, and waits for the word.
thread_local bool g_check_finite = true;

struct OutArray {
    const float* f;
    const double* d;
    long long n;
    const char* what;
};

int check_finite(unsigned* flag, hipStream_t s, std::initializer_list<OutArray> outs)
{
    if (!g_check_finite)
        return STRIDE_OK;
    launch_fill(reinterpret_cast<float*>(flag), 1, 0.f, s);
    unsigned bit = 1;
    for (const OutArray& o : outs) {
        if (o.n > 0 && o.f)
            launch_finite_scan(o.f, o.n, flag, bit, s);
        else if (o.n > 0 && o.d)
            launch_finite_scan(o.d, o.n, flag, bit, s);
        bit <<= 1;
    }
    unsigned host = 0;
    HIP_TRY(hipMemcpyAsync(&host, flag, sizeof(host), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!host)
        return STRIDE_OK;
    std::string names;
    bit = 1;
    for (const OutArray& o : outs) {
        if (host & bit)
            names += names.empty() ? o.what : std::string(", ") + o.what;
        bit <<= 1;
    }
    return fail(STRIDE_E_NONFINITE, "non-finite values in the output: %s", names.c_str());
}

// Flag word of the non-finite check: word 4 of a workspace's scratch
// (words 0-3 hold the vp and medium checks).
unsigned* finite_flag(void* ws) { return reinterpret_cast<unsigned*>(ws) + 4; }

long long phys_points(const stride_plan& P)
{
    long long n = 1;
    for (int a = 0; a < P.nd; ++a)
        n *= P.g.shape[a];
    return n;
}

// The fields of a plan that workspace sizes and gradient paths depend on,
// without the device tables (host only).
void geometry_free_plan(const stride_grid_t* grid, int nrec, stride_plan& P)
{
    P.g = *grid;
    P.nd = grid->ndim;
    P.nt = grid->nt;
    P.torder = grid->time_order == 4 ? 4 : 2;
    P.boundary = grid->boundary;
    P.nrec = nrec;
    P.nb = grid->sponge_cells;
    Dims& d = P.dims;
    d.nd = P.nd;
    for (int a = 0; a < 3; ++a)
        d.n[a] = a < P.nd ? (int)(grid->shape[a] + 2LL * P.nb) : 1;
    int align = pitch_align();
    long long pitch = round_up(d.n[P.nd - 1], align);
    d.total = P.nd == 2 ? (long long)d.n[0] * pitch : (long long)d.n[0] * d.n[1] * pitch;
}

// ------------------------------------------------------------ executors

// Runs a checkpointed gradient on one stream.  forward_phase launches the
// forward sweep up to the first adjoint step (recording traces: the first
// sweep visits every index once); with run = false it only replays the
// bookkeeping, which stride_backward uses to find the pool state the forward
// sweep left behind.  backward_phase launches recomputation and adjoint steps.
// One launch advances one step, so steps and launches count alike.
struct Runner {
    const stride_plan& P;
    GradWs& W;
    hipStream_t s;
    const float* wavelet;
    StepCursor cursor;
    long long steps = 0;         // forward steps
    long long launches = 0;      // forward step launches
    long long adj_steps = 0;     // adjoint steps
    long long adj_launches = 0;  // adjoint step launches
    // Full history, second order: the forward keeps v^n = L u^n + S^n (pool
    // field n) instead of the states, u rotates in the adjoint fields (free
    // until the adjoint starts), and the adjoint images from v^m pointwise
    // instead of a second stencil of u^m.  The same arithmetic as the
    // checkpointed path, so the results are the same bits.
    bool vpath = false;

    // Segmented history (when not every state fits and the cost model of
    // grad_path prefers it): the forward sweep stores the states at the
    // starts of the segments and v^n (fourth order: p^n) over the last
    // segment; the adjoint takes the segments last to first, recomputing a
    // segment's v^n (p^n) from its stored start state (the first from
    // x_0 = 0) just before its adjoint steps, and then runs the full-history
    // path's adjoint steps.  Every step before the last segment is recomputed
    // once; in exchange each second-order adjoint step has one stencil field
    // instead of two, and each fourth-order one two launches instead of
    // three.  The same arithmetic, so the same bits.
    bool segpath = false;
    GradPath path;

    Runner(const stride_plan& p, GradWs& w, hipStream_t st, const float* wav)
        : P(p), W(w), s(st), wavelet(wav), cursor(p.nt, w.snaps, w.peak),
          path(grad_path(p, (long long)w.pool.size(), w.snaps))
    {
        vpath = path.kind == GradPath::kFull && P.torder == 2;
        ppath = path.kind == GradPath::kFull && P.torder == 4;
        segpath = path.kind == GradPath::kSegmented;
    }

    // pool layout of the segmented path: v buffer [0, vbuf), two working
    // fields, then the start state (u^j, u^{j-1}) of segments 1 .. K-2
    float* seg_work(int i) const { return W.pool[path.vbuf + i]; }
    float* seg_state(int k, int i) const { return W.pool[path.vbuf + 2 * k + i]; }

    // One forward step A = u^n, B = u^{n-1} -> C = u^{n+1} (C may be B); with
    // V it also keeps v^n there (kStepV), or with fourth-order time writes its
    // p^n = k (L u^n + St^n) there instead of the scratch p.
    void seg_step(const float* A, const float* B, float* C, int n, float* V, float* traces)
    {
        StepParams p = base_params(P);
        p.A = A;
        p.K = W.k;
        p.step = n;
        p.inj_sig = wavelet;
        if (traces)
            p.smp = rec_samples(P, traces);
        ++steps;
        if (P.torder == 4) {
            float* pp = V ? V : W.p;
            p.C = pp;
            launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, p, s);
            StepParams q = base_params(P);
            q.A = pp;
            q.D = A;
            q.B = B;
            q.C = C;
            q.K = W.k;
            q.step = n;
            launch_step_mode(P.dims, P.R, false, kCorrect, P.cf, P.sp, P.ls_fwd, q, s);
            launches += 2;
            return;
        }
        p.B = B;
        p.C = C;
        if (V) {
            p.V = V;
            launch_step_mode(P.dims, P.R, false, kStepV, P.cf, P.sp, P.ls_fwd, p, s);
        } else {
            launch_step(P.dims, P.R, false, P.cf, P.sp, P.ls_fwd, p, s);
        }
        ++launches;
    }

    // Forward sweep of the segmented path (u rotates in the adjoint fields);
    // returns the field of u^{nt-1}.
    const float* forward_seg(float* traces)
    {
        const int last = path.starts.back();
        launch_fill(W.w[0], P.dims.total, 0.f, s);
        launch_fill(W.w[1], P.dims.total, 0.f, s);
        float *fc = W.w[0], *fp = W.w[1];
        for (int n = 0; n < P.nt - 1; ++n) {
            float* C = seg_sweep_out(path, W.pool, W.w, fc, fp, n + 1);
            seg_step(fc, fp, C, n, n >= last ? W.pool[n - last] : nullptr, traces);
            fp = fc;
            fc = C;
        }
        // v^{nt-1} is held at zero, as on the full-history path
        launch_fill(W.pool[P.nt - 1 - last], P.dims.total, 0.f, s);
        return fc;
    }

    // Adjoint steps e-1 .. j with v^m in V[m - j] (imaging in pairs as in
    // backward_v; segment ends other than nt are even, so a pair never
    // straddles two segments).
    void adjoint_v(int j, int e, float* const* V, int& wa, const float* grad_traces,
                   float* dwavelet)
    {
        if (P.torder == 4) {
            adjoint_p(j, e, V, wa, grad_traces, dwavelet);
            return;
        }
        for (int m = e - 1; m >= j; --m) {
            const bool image = (m % 2) == 0;
            StepParams p = base_params(P);
            p.A = W.w[wa];
            p.B = W.w[1 - wa];
            p.C = W.w[1 - wa];
            p.K = W.k;
            p.G = W.G;
            p.V = V[m - j];
            p.V2 = m + 1 < e ? V[m + 1 - j] : nullptr;
            p.step = m;
            p.inj = P.rec_inj_v;
            p.inj_sig = grad_traces;
            p.inj_stride = P.nt;
            p.img = P.no_inj;
            if (dwavelet)
                p.smp = src_samples(P, dwavelet);
            launch_step_mode(P.dims, P.R, true, image ? kImageV : kAdjPlain, P.cf, P.sp, P.ls_adjv, p,
                             s);
            ++adj_steps;
            ++adj_launches;
            wa = 1 - wa;
        }
    }

    void backward_seg(const float* grad_traces, float* dwavelet)
    {
        const std::vector<int>& j = path.starts;
        const int K = (int)j.size();
        int wa = 0;
        for (int k = K - 1; k >= 0; --k) {
            const int e = k + 1 < K ? j[k + 1] : P.nt;
            if (k < K - 1) {
                // recompute v^n, n in [j_k, e), from the segment's start state
                float* fc = k >= 1 ? seg_state(k, 0) : seg_work(0);
                float* fp = k >= 1 ? seg_state(k, 1) : seg_work(1);
                if (k == 0) {
                    launch_fill(fc, P.dims.total, 0.f, s);
                    launch_fill(fp, P.dims.total, 0.f, s);
                }
                const int seg = g_timer.begin(s);
                const long long s0 = steps, l0 = launches;
                for (int n = j[k]; n < e; ++n) {
                    seg_step(fc, fp, fp, n, W.pool[n - j[k]], nullptr);
                    std::swap(fc, fp);
                }
                g_timer.end(seg, s, 2, steps - s0, launches - l0);
            }
            adjoint_v(j[k], e, W.pool.data(), wa, grad_traces, dwavelet);
        }
    }

    // Full history, fourth order: the forward's first launch writes p^n =
    // k (L u^n + St^n) into history field n (where the checkpointed path
    // writes scratch), u rotates in the adjoint fields, and the adjoint takes
    // p^m from the history instead of recomputing it: two launches per adjoint
    // step instead of three, the same bits.
    bool ppath = false;

    const float* forward_p(float* traces)
    {
        float* u[2] = {W.w[0], W.w[1]};
        launch_fill(u[0], P.dims.total, 0.f, s);
        launch_fill(u[1], P.dims.total, 0.f, s);
        int cur = 0;
        for (int n = 0; n < P.nt - 1; ++n) {
            StepParams p = base_params(P);
            p.A = u[cur];
            p.C = W.pool[n];
            p.K = W.k;
            p.step = n;
            p.inj_sig = wavelet;
            if (traces)
                p.smp = rec_samples(P, traces);
            launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, p, s);
            StepParams q = base_params(P);
            q.A = W.pool[n];
            q.D = u[cur];
            q.B = u[1 - cur];
            q.C = u[1 - cur];
            q.K = W.k;
            q.step = n;
            launch_step_mode(P.dims, P.R, false, kCorrect, P.cf, P.sp, P.ls_fwd, q, s);
            cur = 1 - cur;
        }
        // p^{nt-1} is never formed; the adjoint step at nt-1 multiplies it by
        // w^{nt} = 0 (and q = k L w^{nt} = 0), so it is held at zero
        launch_fill(W.pool[P.nt - 1], P.dims.total, 0.f, s);
        steps += P.nt - 1;
        launches += 2LL * (P.nt - 1);
        return u[cur];
    }

    void backward_p(const float* grad_traces, float* dwavelet)
    {
        int wa = 0;
        adjoint_p(0, P.nt, W.pool.data(), wa, grad_traces, dwavelet);
    }

    // Fourth-order adjoint steps e-1 .. j with p^m = Pm[m - j] kept: q = k L
    // w^{m+1}, then the correction (two launches instead of three).
    void adjoint_p(int j, int e, float* const* Pm, int& wa, const float* grad_traces,
                   float* dwavelet)
    {
        for (int m = e - 1; m >= j; --m) {
            StepParams q = base_params(P);
            q.A = W.w[wa];
            q.C = W.q;
            q.K = W.k;
            q.step = m;
            q.inj = P.no_inj;
            if (dwavelet)
                q.smp = src_samples(P, dwavelet);
            launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, q, s);
            StepParams c = base_params(P);
            c.A = W.q;
            c.U = Pm[m - j];
            c.D = W.w[wa];
            c.B = W.w[1 - wa];
            c.C = W.w[1 - wa];
            c.K = W.k;
            c.G = W.G;
            c.step = m;
            c.inj = P.rec_inj;
            c.inj_sig = grad_traces;
            c.inj_stride = P.nt;
            c.img = P.no_inj;
            if (dwavelet) {
                c.smp = src_samples(P, dwavelet);
                c.smp.scale = 1.f / 12.f;
                c.smp.accumulate = 1;
            }
            launch_step_mode(P.dims, P.R, true, kCorrect, P.cf, P.sp, P.ls_adj, c, s);
            ++adj_steps;
            adj_launches += 2;
            wa = 1 - wa;
        }
    }

    // Forward sweep of the full-history path; returns the field of u^{nt-1}.
    const float* forward_v(float* traces)
    {
        float* u[2] = {W.w[0], W.w[1]};
        launch_fill(u[0], P.dims.total, 0.f, s);
        launch_fill(u[1], P.dims.total, 0.f, s);
        int cur = 0;
        for (int n = 0; n < P.nt - 1; ++n) {
            StepParams p = base_params(P);
            p.A = u[cur];
            p.B = u[1 - cur];
            p.C = u[1 - cur];
            p.K = W.k;
            p.V = W.pool[n];
            p.step = n;
            p.inj_sig = wavelet;
            if (traces)
                p.smp = rec_samples(P, traces);
            launch_step_mode(P.dims, P.R, false, kStepV, P.cf, P.sp, P.ls_fwd, p, s);
            cur = 1 - cur;
        }
        // v^{nt-1} is never formed (no step leaves u^{nt-1}); the adjoint step
        // at nt-1 multiplies it by w^{nt} = 0, so it is held at zero
        launch_fill(W.pool[P.nt - 1], P.dims.total, 0.f, s);
        steps += P.nt - 1;
        launches += P.nt - 1;
        return u[cur];
    }

    // Imaging terms in pairs: an odd step m+1 leaves G alone (kAdjPlain), the
    // even step m after it adds both, G = fma(w^{m+1}, v^m, fma(w^{m+2}, v^{m+1}, G)),
    // the same operations in the same order as one term per step, with G read
    // and written every other step.
    void backward_v(const float* grad_traces, float* dwavelet)
    {
        int wa = 0;
        adjoint_v(0, P.nt, W.pool.data(), wa, grad_traces, dwavelet);
    }

    void fwd_launch(const StepOp& op, float* traces)
    {
        StepParams p = base_params(P);
        p.A = W.pool[op.a];
        p.B = W.pool[op.b];
        p.C = W.pool[op.c];
        p.K = W.k;
        p.step = op.step;
        p.inj_sig = wavelet;
        if (traces && op.first_sweep)
            p.smp = rec_samples(P, traces);
        ++steps;
        if (P.torder == 4) {
            // p = k (L u^n + St^n), then u^{n+1} from the stencil of p
            StepParams q = p;
            p.C = W.p;
            launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, p, s);
            q.A = W.p;
            q.D = W.pool[op.a];
            q.smp = SampleSet{};
            launch_step_mode(P.dims, P.R, false, kCorrect, P.cf, P.sp, P.ls_fwd, q, s);
            launches += 2;
            return;
        }
        launch_step(P.dims, P.R, false, P.cf, P.sp, P.ls_fwd, p, s);
        ++launches;
    }

    // Fourth-order adjoint step m: p = k (L u^m + St^m) and q = k L w^{m+1}
    // (no injection: the empty table), then w^m and the imaging update.
    void adj4_launch(const StepOp& op, int wa, const float* grad_traces, float* dwavelet)
    {
        StepParams p = base_params(P);
        p.A = W.pool[op.a];
        p.C = W.p;
        p.K = W.k;
        p.step = op.step;
        p.inj_sig = wavelet;
        launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, p, s);
        StepParams q = base_params(P);
        q.A = W.w[wa];
        q.C = W.q;
        q.K = W.k;
        q.step = op.step;
        q.inj = P.no_inj;
        // wavelet cotangent before the time filter: W_s (w + q/12) / cell volume,
        // the w part sampled here, the q part added by the correction launch
        if (dwavelet)
            q.smp = src_samples(P, dwavelet);
        launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, q, s);
        StepParams c = base_params(P);
        c.A = W.q;
        c.U = W.p;
        c.D = W.w[wa];
        c.B = W.w[1 - wa];
        c.C = W.w[1 - wa];
        c.K = W.k;
        c.G = W.G;
        c.step = op.step;
        c.inj = P.rec_inj;
        c.inj_sig = grad_traces;
        c.inj_stride = P.nt;
        c.img = P.no_inj;
        if (dwavelet) {
            c.smp = src_samples(P, dwavelet);
            c.smp.scale = 1.f / 12.f;
            c.smp.accumulate = 1;
        }
        launch_step_mode(P.dims, P.R, true, kCorrect, P.cf, P.sp, P.ls_adj, c, s);
        adj_launches += 3;
    }

    void forward_phase(bool run, float* traces)
    {
        StepOp op;
        while (cursor.next(op)) {
            if (op.reverse) {
                cursor.unget(op);
                return;
            }
            if (run)
                fwd_launch(op, traces);
        }
    }

    void backward_phase(const float* grad_traces, float* dwavelet)
    {
        int wa = 0;   // W.w[wa] = w^{m+1}, W.w[1-wa] = w^{m+2}
        int seg = -1;
        long long seg_steps = 0, seg_launches = 0;
        StepOp op;
        while (cursor.next(op)) {
            if (!op.reverse) {
                if (seg < 0) {
                    seg = g_timer.begin(s);
                    seg_steps = steps;
                    seg_launches = launches;
                }
                fwd_launch(op, nullptr);
                continue;
            }
            if (seg >= 0) {
                g_timer.end(seg, s, 2, steps - seg_steps, launches - seg_launches);
                seg = -1;
            }
            ++adj_steps;
            if (P.torder == 4) {
                adj4_launch(op, wa, grad_traces, dwavelet);
                wa = 1 - wa;
                continue;
            }
            StepParams p = base_params(P);
            p.A = W.w[wa];
            p.B = W.w[1 - wa];
            p.C = W.w[1 - wa];
            p.K = W.k;
            p.U = W.pool[op.a];
            p.G = W.G;
            p.step = op.step;
            p.inj = P.rec_inj;
            p.inj_sig = grad_traces;
            p.inj_stride = P.nt;
            p.img = P.src_img;
            p.img_sig = wavelet;
            p.img_stride = P.nt;
            if (dwavelet)
                p.smp = src_samples(P, dwavelet);
            launch_step(P.dims, P.R, true, P.cf, P.sp, P.ls_adj, p, s);
            ++adj_launches;
            wa = 1 - wa;
        }
        if (seg >= 0)
            g_timer.end(seg, s, 2, steps - seg_steps, launches - seg_launches);
    }
};

int forward_solve(const stride_plan& P, const float* vp, const float* wavelet, float* traces,
                  void* ws, size_t bytes, hipStream_t s)
{
    if (!vp || (!wavelet && P.nsrc > 0) || (!traces && P.nrec > 0))
        return fail(STRIDE_E_INVALID_ARG, "vp, wavelet and traces must be device pointers");
    FwdWs F;
    int rc = fwd_ws(P, ws, bytes, F);
    if (rc)
        return rc;
    float* k = F.k;
    float* const* u = F.u;
    rc = check_vp(P, vp, F.flags, s);
    if (rc)
        return rc;
    launch_prep_k(P.dims, vp, P.g.dt, k, s);
    launch_fill(u[0], P.dims.total, 0.f, s);
    launch_fill(u[1], P.dims.total, 0.f, s);
    int tid = g_timer.begin(s);
    int cur = 0;
    if (P.torder == 4) {
        // two launches per step: p = k (L u + St) (sampling u^n), then the
        // corrected update from the stencil of p
        for (int n = 0; n < P.nt - 1; ++n) {
            StepParams p = base_params(P);
            p.A = u[cur];
            p.C = F.p;
            p.K = k;
            p.step = n;
            p.inj_sig = wavelet;
            p.smp = rec_samples(P, traces);
            launch_step_mode(P.dims, P.R, false, kPrep, P.cf, P.sp, P.ls_fwd, p, s);
            StepParams q = base_params(P);
            q.A = F.p;
            q.D = u[cur];
            q.B = u[1 - cur];
            q.C = u[1 - cur];
            q.K = k;
            q.step = n;
            launch_step_mode(P.dims, P.R, false, kCorrect, P.cf, P.sp, P.ls_fwd, q, s);
            cur = 1 - cur;
        }
        g_timer.end(tid, s, 0, P.nt - 1, 2LL * (P.nt - 1));
        launch_sample(rec_samples(P, traces), u[cur], P.nt - 1, s);
        HIP_TRY(hipGetLastError());
        return check_finite(finite_flag(ws), s, {{traces, nullptr, (long long)P.nrec * P.nt, "traces"}});
    }
    PmlParams pm{};
    int ps = 0;
    if (P.boundary == 1) {
        for (int a = 0; a < P.nd; ++a) {
            launch_fill(F.psi[0][a], P.dims.total, 0.f, s);
            launch_fill(F.psi[1][a], P.dims.total, 0.f, s);
            launch_fill(F.chi[a], P.dims.total, 0.f, s);
            pm.chi[a] = F.chi[a];
            pm.c0[a] = P.pml_c0[a];
            pm.zmax[a] = P.pml_zmax[a];
        }
        pm.k = k;
        pm.dt = (float)P.g.dt;
    }
    for (int n = 0; n < P.nt - 1; ++n) {
        StepParams p = base_params(P);
        p.A = u[cur];
        p.B = u[1 - cur];
        p.C = u[1 - cur];
        p.K = k;
        p.step = n;
        p.inj_sig = wavelet;
        p.smp = rec_samples(P, traces);
        launch_step(P.dims, P.R, false, P.cf, P.sp, P.ls_fwd, p, s);
        if (P.boundary == 1) {
            // the step above wrote the undamped leapfrog; u^n is still intact
            pm.u = u[cur];
            pm.un = u[1 - cur];
            for (int a = 0; a < P.nd; ++a) {
                pm.psi[a] = F.psi[ps][a];
                pm.psin[a] = F.psi[1 - ps][a];
            }
            launch_pml_correction(P.dims, P.R, P.cf, pm, s);
            ps = 1 - ps;
        }
        cur = 1 - cur;
    }
    g_timer.end(tid, s, 0, P.nt - 1, (P.boundary == 1 ? 2LL : 1LL) * (P.nt - 1));
    launch_sample(rec_samples(P, traces), u[cur], P.nt - 1, s);
    HIP_TRY(hipGetLastError());
    return check_finite(finite_flag(ws), s, {{traces, nullptr, (long long)P.nrec * P.nt, "traces"}});
}

// Forward solve in a heterogeneous medium: three rotating wavefields (the
// step reads u^{n-1} as a stencil field, so u^{n+1} cannot overwrite it), the
// medium fields prepared once, one kMedium launch per step on the two-field
// launch shape (whose source table is src_img).
// Views of a medium workspace: [scratch | k | u0 | u1 | u2 | gamma_a x nd | att]
// (the gradient adds [G | traces | residual | H x (nt - 1)]).
struct MediumWs {
    unsigned* flags;
    float* k;
    float* u[3];
    float* gam[3];
    float* att;
    char* tail;
};

void medium_views(const stride_plan& P, const Layout& L, void* ws, MediumWs& M)
{
    char* b = (char*)ws;
    M.flags = (unsigned*)b;
    b += L.scratch;
    M.k = (float*)b;
    b += L.field;
    for (int i = 0; i < 3; ++i, b += L.field)
        M.u[i] = (float*)b;
    for (int a = 0; a < 3; ++a)
        M.gam[a] = nullptr;
    for (int a = 0; a < P.nd; ++a, b += L.field)
        M.gam[a] = (float*)b;
    M.att = (float*)b;
    M.tail = b + L.field;
}

int medium_args(const stride_plan& P, const float* vp, const float* wavelet, int att_power)
{
    if (!vp || (!wavelet && P.nsrc > 0))
        return fail(STRIDE_E_INVALID_ARG, "vp and wavelet must be device pointers");
    if (P.torder != 2)
        return fail(STRIDE_E_INVALID_ARG, "medium solves need time_order 2");
    if (P.boundary == 1)
        return fail(STRIDE_E_INVALID_ARG, "medium solves use the sponge, not the PML");
    if (att_power != 0 && att_power != 2)
        return fail(STRIDE_E_INVALID_ARG, "att_power must be 0 or 2 (got %d)", att_power);
    return STRIDE_OK;
}

// Value and stability checks of a medium solve (one stream sync), then k and
// the medium fields on the padded grid.
int prepare_medium(const stride_plan& P, const float* vp, const float* rho, const float* alpha0,
                   int att_power, const MediumWs& M, hipStream_t s)
{
    const long long nphys = phys_points(P);
    launch_vp_check(vp, nphys, M.flags, s);
    launch_medium_check(vp, rho, alpha0, nphys, att_power, P.g.dt, M.flags, s);
    unsigned host[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(host, M.flags, sizeof(host), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (host[1])
        return fail(STRIDE_E_INVALID_ARG, "vp contains non-positive or non-finite values");
    if (host[2])
        return fail(STRIDE_E_INVALID_ARG,
                    "rho must be positive and finite, alpha0 non-negative and finite");
    float vmax, veff2;
    std::memcpy(&vmax, &host[0], sizeof(float));
    std::memcpy(&veff2, &host[3], sizeof(float));
    // with y = 2 the limit is on vp^2 (1 + 2 beta) (frozen coefficients)
    int rc = check_cfl(P, std::max((double)vmax, std::sqrt((double)veff2)));
    if (rc)
        return rc;
    float* gam[3] = {M.gam[0], M.gam[1], M.gam[2]};
    launch_prep_k(P.dims, vp, P.g.dt, M.k, s);
    launch_prep_medium(P.dims, P.fd1, vp, rho, alpha0, att_power, P.g.dt, gam, M.att, s);
    return STRIDE_OK;
}

// Medium forward sweep: three rotating wavefields (the step reads u^{n-1} as a
// stencil field, so u^{n+1} cannot overwrite it), one kMedium launch per step
// on the two-field launch shape (whose source table is src_img); with H the
// step n also stores its imaging factor into H[n].  Returns the field of u^{nt-1}.
const float* medium_sweep(const stride_plan& P, const MediumWs& M, const float* wavelet,
                          int att_power, float* traces, float* const* H, hipStream_t s)
{
    launch_fill(M.u[0], P.dims.total, 0.f, s);
    launch_fill(M.u[1], P.dims.total, 0.f, s);
    int tid = g_timer.begin(s);
    int cur = 0, prev = 1, next = 2;
    for (int n = 0; n < P.nt - 1; ++n) {
        StepParams p = base_params(P);
        p.A = M.u[cur];
        p.B = M.u[prev];
        p.C = M.u[next];
        p.K = M.k;
        p.step = n;
        p.inj = P.src_img;
        p.inj_sig = wavelet;
        p.smp = rec_samples(P, traces);
        for (int a = 0; a < 3; ++a)
            p.gam[a] = M.gam[a] ? M.gam[a] : M.gam[0];
        p.att = M.att;
        p.att_power = att_power;
        p.V = H ? H[n] : nullptr;
        launch_step_mode(P.dims, P.R, false, kMedium, P.cf, P.sp, P.ls_adj, p, s);
        const int t = prev;
        prev = cur;
        cur = next;
        next = t;
    }
    g_timer.end(tid, s, 0, P.nt - 1, P.nt - 1);
    launch_sample(rec_samples(P, traces), M.u[cur], P.nt - 1, s);
    return M.u[cur];
}

int forward_medium(const stride_plan& P, const float* vp, const float* rho, const float* alpha0,
                   int att_power, const float* wavelet, float* traces, void* ws, size_t bytes,
                   hipStream_t s)
{
    int rc = medium_args(P, vp, wavelet, att_power);
    if (rc)
        return rc;
    if (!traces && P.nrec > 0)
        return fail(STRIDE_E_INVALID_ARG, "traces must be a device pointer");
    Layout L = layout_of(P);
    if (!ws || (uintptr_t)ws % 256)
        return fail(STRIDE_E_INVALID_ARG, "workspace must be a 256-byte aligned device pointer");
    if (bytes < L.medium)
        return fail(STRIDE_E_WORKSPACE, "medium forward workspace needs %zu bytes (got %zu)",
                    L.medium, bytes);
    MediumWs M;
    medium_views(P, L, ws, M);
    if ((rc = prepare_medium(P, vp, rho, alpha0, att_power, M, s)))
        return rc;
    medium_sweep(P, M, wavelet, att_power, traces, nullptr, s);
    HIP_TRY(hipGetLastError());
    return check_finite(finite_flag(ws), s, {{traces, nullptr, (long long)P.nrec * P.nt, "traces"}});
}

// Shot gradient in the medium: the medium sweep storing every step's imaging
// factor H (or, in a smaller workspace, checkpointed states from which h^m is
// recomputed just before it is needed), residual and misfit, then per adjoint
// step the direct medium adjoint kernel (w rotates through three wavefields)
// and the receiver residual injected through the plan's table.
int gradient_medium(const stride_plan& P, const float* vp, const float* rho, const float* alpha0,
                    int att_power, const float* wavelet, const float* observed, float* traces,
                    double* misfit, float* dvp, void* ws, size_t bytes, hipStream_t s)
{
    int rc = medium_args(P, vp, wavelet, att_power);
    if (rc)
        return rc;
    if ((!observed && P.nrec > 0) || !misfit || !dvp)
        return fail(STRIDE_E_INVALID_ARG, "observed, misfit and dvp must be device pointers");
    Layout L = layout_of(P);
    if (!ws || (uintptr_t)ws % 256)
        return fail(STRIDE_E_INVALID_ARG, "workspace must be a 256-byte aligned device pointer");
    // every step's imaging factor kept, or checkpointed forward states (the
    // medium step reads u^{n-1} as a stencil field, so steps never write in
    // place) with h^m recomputed from x_m before adjoint step m
    const bool full = bytes >= L.grad_medium;
    if (!full && bytes < L.grad_medium_fixed + 5 * L.field)
        return fail(STRIDE_E_WORKSPACE,
                    "medium gradient workspace needs %zu bytes (every imaging factor kept) or at "
                    "least %zu (checkpointed), got %zu", L.grad_medium,
                    L.grad_medium_fixed + 5 * L.field, bytes);
    MediumWs M;
    medium_views(P, L, ws, M);
    char* b = M.tail;
    float* G = (float*)b;
    b += L.field;
    float* tr_ws = (float*)b;
    b += L.traces;
    float* residual = (float*)b;
    b += L.traces;
    std::vector<float*> H, pool;
    float *hbuf = nullptr, *cbuf = nullptr;
    std::unique_ptr<StepCursor> cursor;
    // segmented history (as for the plain gradient): h^n over the last
    // segment kept by the first sweep, each other segment's h^n recomputed
    // once from its start state; pool = h buffer [0, hlen), working pair,
    // start state of segment k at hlen + 2k; preferred whenever it fits, since
    // it saves the binomial path's recomputation of h^m at every adjoint step
    bool seg = false;
    std::vector<int> segs;
    int hlen = 0;
    if (full) {
        H.resize((size_t)std::max(P.nt - 1, 1));
        for (int n = 0; n < P.nt - 1; ++n, b += L.field)
            H[n] = (float*)b;
    } else {
        hbuf = (float*)b;
        b += L.field;
        cbuf = (float*)b;
        b += L.field;
        const long long nf = (long long)((bytes - L.grad_medium_fixed) / L.field);
        for (long long f = 0; f < nf; ++f, b += L.field)
            pool.push_back((float*)b);
        seg = make_segments(P.nt, nf, segs, hlen);
        if (!seg) {
            const int snaps = snaps_for_fields(P.nt, nf - 1);
            if (snaps < 0)
                return fail(STRIDE_E_WORKSPACE,
                            "medium gradient workspace too small for checkpointing");
            cursor = std::make_unique<StepCursor>(P.nt, snaps, (int)nf, false);
        }
    }
    if ((rc = prepare_medium(P, vp, rho, alpha0, att_power, M, s)))
        return rc;
    float* tr = traces ? traces : tr_ws;
    // one medium step u^n = A, u^{n-1} = B -> C, sampling into smp, h into V
    auto medium_step = [&](const float* A, const float* B, float* C, int n, float* smp, float* V) {
        StepParams p = base_params(P);
        p.A = A;
        p.B = B;
        p.C = C;
        p.K = M.k;
        p.step = n;
        p.inj = P.src_img;
        p.inj_sig = wavelet;
        if (smp)
            p.smp = rec_samples(P, smp);
        for (int a = 0; a < 3; ++a)
            p.gam[a] = M.gam[a] ? M.gam[a] : M.gam[0];
        p.att = M.att;
        p.att_power = att_power;
        p.V = V;
        launch_step_mode(P.dims, P.R, false, kMedium, P.cf, P.sp, P.ls_adj, p, s);
    };
    // the field of three that is neither a nor b
    auto third = [](float* const* f3, const float* a, const float* b3) {
        for (int i = 0; i < 3; ++i)
            if (f3[i] != a && f3[i] != b3)
                return f3[i];
        return (float*)nullptr;
    };
    if (full) {
        medium_sweep(P, M, wavelet, att_power, tr, H.data(), s);
    } else if (seg) {
        // u rotates through the three wavefields (free until the adjoint);
        // the start states x_{j_k} (k = 1 .. K-2) are written into their pool
        // pair by the steps that produce them
        const int K = (int)segs.size(), last = segs.back();
        launch_fill(M.u[0], P.dims.total, 0.f, s);
        launch_fill(M.u[1], P.dims.total, 0.f, s);
        float *fc = M.u[0], *fp = M.u[1];
        int tid = g_timer.begin(s);
        for (int n = 0; n < P.nt - 1; ++n) {
            float* out = nullptr;
            for (int k = 1; k + 1 < K && !out; ++k)
                out = n + 1 == segs[k] ? pool[hlen + 2 * k]
                      : n + 1 == segs[k] - 1 ? pool[hlen + 2 * k + 1] : nullptr;
            if (!out)
                out = third(M.u, fc, fp);
            medium_step(fc, fp, out, n, tr, n >= last ? pool[n - last] : nullptr);
            fp = fc;
            fc = out;
        }
        g_timer.end(tid, s, 0, P.nt - 1, P.nt - 1);
        launch_sample(rec_samples(P, tr), fc, P.nt - 1, s);
    } else {
        launch_fill(pool[0], P.dims.total, 0.f, s);
        launch_fill(pool[1], P.dims.total, 0.f, s);
        int tid = g_timer.begin(s);
        long long fsteps = 0;
        StepOp op;
        while (cursor->next(op)) {
            if (op.reverse) {
                cursor->unget(op);
                break;
            }
            medium_step(pool[op.a], pool[op.b], pool[op.c], op.step, op.first_sweep ? tr : nullptr,
                        nullptr);
            ++fsteps;
        }
        g_timer.end(tid, s, 0, fsteps, fsteps);
        if (cursor->overflow())
            return fail(STRIDE_E_WORKSPACE, "checkpoint pool overflow");
        launch_sample(rec_samples(P, tr), pool[cursor->cur()], P.nt - 1, s);
    }
    const long long ntr = (long long)P.nrec * P.nt;
    launch_residual_misfit(tr, observed, residual, ntr, misfit, (double*)(M.flags + 64), s);

    // adjoint: w^{m+1} and w^{m+2} start at zero; step m images with h^m
    float* w[3] = {M.u[0], M.u[1], M.u[2]};
    for (int i = 0; i < 3; ++i)
        launch_fill(w[i], P.dims.total, 0.f, s);
    launch_fill(G, P.dims.total, 0.f, s);
    int i0 = 0, i1 = 1, i2 = 2;   // w^m, w^{m+1}, w^{m+2}
    auto adjoint_step = [&](int m, const float* Hm) {
        MediumAdjParams mp{};
        mp.w1 = w[i1];
        mp.w2 = w[i2];
        mp.w0 = w[i0];
        mp.k = M.k;
        for (int a = 0; a < 3; ++a)
            mp.gam[a] = M.gam[a] ? M.gam[a] : M.gam[0];
        mp.att = M.att;
        mp.att_power = att_power;
        mp.H = Hm;    // w^{nt} = 0: step nt-1 images nothing
        mp.G = G;
        launch_medium_adjoint(P.dims, P.R, P.cf, P.sp, mp, s);
        if (m == 0)
            return;   // w^0 is not needed; the launch above added the last imaging term
        launch_inject_table(P.dims, P.ls_adj, P.rec_inj, residual, P.nt, m, M.k, M.att, att_power,
                            P.sp, w[i0], s);
        const int t = i2;
        i2 = i1;
        i1 = i0;
        i0 = t;
    };
    int tid = g_timer.begin(s);
    long long alaunches = 2LL * P.nt - 1;   // adjoint step + receiver injection (none at m = 0)
    if (full) {
        for (int m = P.nt - 1; m >= 0; --m)
            adjoint_step(m, m <= P.nt - 2 ? H[m] : nullptr);
    } else if (seg) {
        const int K = (int)segs.size();
        for (int k = K - 1; k >= 0; --k) {
            const int j = segs[k], e = k + 1 < K ? segs[k + 1] : P.nt;
            if (k < K - 1) {
                // h^n, n in [j, e), from the segment's start state (x_0 = 0 in
                // the working pair for the first); the scratch field is the third
                float* f3[3] = {pool[hlen + 2 * k], pool[hlen + 2 * k + 1], cbuf};
                if (k == 0) {
                    launch_fill(f3[0], P.dims.total, 0.f, s);
                    launch_fill(f3[1], P.dims.total, 0.f, s);
                }
                float *fc = f3[0], *fp = f3[1];
                for (int n = j; n < e; ++n) {
                    float* out = third(f3, fc, fp);
                    medium_step(fc, fp, out, n, nullptr, pool[n - j]);
                    fp = fc;
                    fc = out;
                    ++alaunches;
                }
            }
            for (int m = e - 1; m >= j; --m)
                adjoint_step(m, m <= P.nt - 2 ? pool[m - j] : nullptr);
        }
    } else {
        StepOp op;
        while (cursor->next(op)) {
            ++alaunches;
            if (!op.reverse) {
                medium_step(pool[op.a], pool[op.b], pool[op.c], op.step, nullptr, nullptr);
                continue;
            }
            const int m = op.step;
            if (m <= P.nt - 2)   // h^m from x_m = (u^m, u^{m-1}); u^{m+1} is discarded
                medium_step(pool[op.a], pool[op.b], cbuf, m, nullptr, hbuf);
            else
                --alaunches;
            adjoint_step(m, m <= P.nt - 2 ? hbuf : nullptr);
        }
        if (cursor->overflow())
            return fail(STRIDE_E_WORKSPACE, "checkpoint pool overflow");
    }
    g_timer.end(tid, s, 1, P.nt, alaunches);
    // dvp = P^T (2 G / vp_pad); two wavefields serve as the finalise's scratch
    launch_finalize_dvp(P.dims, G, nullptr, vp, dvp, w[i1], w[i2], s);
    HIP_TRY(hipGetLastError());
    return check_finite(finite_flag(ws), s,
                        {{tr, nullptr, ntr, "traces"}, {nullptr, misfit, 1, "misfit"},
                         {dvp, nullptr, phys_points(P), "dvp"}});
}

int forward_save(const stride_plan& P, const float* vp, const float* wavelet, float* traces,
                 void* ws, size_t bytes, hipStream_t s, GradWs& W)
{
    if (!vp || (!wavelet && P.nsrc > 0))
        return fail(STRIDE_E_INVALID_ARG, "vp and wavelet must be device pointers");
    int rc = grad_ws(P, ws, bytes, W);
    if (rc)
        return rc;
    rc = check_vp(P, vp, W.flags, s);
    if (rc)
        return rc;
    float* tr = traces ? traces : W.traces;
    launch_prep_k(P.dims, vp, P.g.dt, W.k, s);
    TraceRange range_("forward sweep");
    Runner run(P, W, s, wavelet);
    const float* last;
    int tid = g_timer.begin(s);
    if (run.vpath || run.ppath || run.segpath) {
        last = run.vpath ? run.forward_v(tr) : run.ppath ? run.forward_p(tr) : run.forward_seg(tr);
        g_timer.end(tid, s, 0, run.steps, run.launches);
    } else {
        launch_fill(W.pool[0], P.dims.total, 0.f, s);
        launch_fill(W.pool[1], P.dims.total, 0.f, s);
        run.forward_phase(true, tr);
        g_timer.end(tid, s, 0, run.steps, run.launches);
        if (run.cursor.overflow())
            return fail(STRIDE_E_WORKSPACE, "checkpoint pool overflow");
        last = W.pool[run.cursor.cur()];
    }
    // last sample from the final state x_{nt-1}
    launch_sample(rec_samples(P, tr), last, P.nt - 1, s);
    if (traces && traces != W.traces)
        launch_copy(W.traces, traces, (long long)P.nrec * P.nt, s);
    HIP_TRY(hipGetLastError());
    return STRIDE_OK;
}

int backward(const stride_plan& P, const float* vp, const float* wavelet, const float* grad_traces,
             float* dvp, float* dwavelet, void* ws, size_t bytes, hipStream_t s)
{
    if (!vp || (!wavelet && P.nsrc > 0) || (!grad_traces && P.nrec > 0) || !dvp)
        return fail(STRIDE_E_INVALID_ARG, "vp, wavelet, grad_traces and dvp must be device pointers");
    if (dwavelet && P.torder == 4 && P.nt > 15360)
        return fail(STRIDE_E_INVALID_ARG,
                    "the fourth-order wavelet gradient filters rows of at most 15360 samples");
    GradWs W;
    int rc = grad_ws(P, ws, bytes, W);
    if (rc)
        return rc;
    Runner run(P, W, s, wavelet);
    if (!run.vpath && !run.ppath && !run.segpath)
        run.forward_phase(false, nullptr);
    launch_fill(W.G, P.dims.total, 0.f, s);
    launch_fill(W.w[0], P.dims.total, 0.f, s);
    launch_fill(W.w[1], P.dims.total, 0.f, s);
    TraceRange range_("adjoint sweep");
    int tid = g_timer.begin(s);
    if (run.vpath)
        run.backward_v(grad_traces, dwavelet);
    else if (run.segpath)
        run.backward_seg(grad_traces, dwavelet);
    else if (run.ppath)
        run.backward_p(grad_traces, dwavelet);
    else
        run.backward_phase(grad_traces, dwavelet);
    g_timer.end(tid, s, 1, run.adj_steps, run.adj_launches);
    if (run.cursor.overflow())
        return fail(STRIDE_E_WORKSPACE, "checkpoint pool overflow");
    if (dwavelet && P.torder == 4)
        launch_time_filter3(dwavelet, P.nsrc, P.nt, s);
    // the fourth-order accumulator holds k G
    launch_finalize_dvp(P.dims, W.G, P.torder == 4 ? W.k : nullptr, vp, dvp, W.w[0], W.w[1], s);
    HIP_TRY(hipGetLastError());
    return STRIDE_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// ------------------------------------------------------------ allocation-free forward
//
// Workspace of stride_plan_forward_static: a file-scope device array that each
// device holds for the life of the process.  On the host, `scratch` names only
// a stand-in for the device copy; every host use goes through the device
// address hipGetSymbolAddress returns, looked up once per device (with that
// device current) and kept.
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[STRIDE_STATIC_WORKSPACE_BYTES];

namespace {

// Device address of `scratch` on the current device.
int static_workspace(void** out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxStaticDevices)
        return fail(STRIDE_E_INVALID_ARG, "device %d is beyond the %d devices the static workspace serves",
                    dev, kMaxStaticDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || (uintptr_t)ptr % 256)
            return fail(STRIDE_E_HIP, "static workspace address %p is not 256-byte aligned", ptr);
        g_static_ptr[dev] = ptr;
    }
    *out = g_static_ptr[dev];
    return STRIDE_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

const char* stride_last_error(void) { return g_err.c_str(); }

const char* stride_error_string(int code)
{
    switch (code) {
    case STRIDE_OK: return "ok";
    case STRIDE_E_INVALID_ARG: return "invalid argument";
    case STRIDE_E_CFL: return "CFL stability limit violated";
    case STRIDE_E_GEOMETRY: return "source or receiver outside the physical grid";
    case STRIDE_E_WORKSPACE: return "workspace too small";
    case STRIDE_E_HIP: return "HIP runtime error";
    case STRIDE_E_NONFINITE: return "non-finite values";
    default: return "unknown error";
    }
}

int stride_plan_create(const stride_grid_t* grid, int32_t nsrc, const double* src_xyz,
                       int32_t nrec, const double* rec_xyz, stride_plan_t** out)
{
    g_err.clear();
    if (!out)
        return fail(STRIDE_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int rc = validate_grid(grid);
    if (rc)
        return rc;
    if (nsrc < 0 || nrec < 0 || (nsrc > 0 && !src_xyz) || (nrec > 0 && !rec_xyz))
        return fail(STRIDE_E_INVALID_ARG, "bad source/receiver arrays");
    stride_plan* P = new stride_plan();
    P->g = *grid;
    P->nd = grid->ndim;
    P->R = grid->space_order / 2;
    P->nb = grid->sponge_cells;
    P->nt = grid->nt;
    P->torder = grid->time_order == 4 ? 4 : 2;
    P->nsrc = nsrc;
    P->ntap = taps_per_point(P->nd, grid->interp);
    P->nrec = nrec;
    P->blob = nullptr;

    Dims& d = P->dims;
    d.nd = P->nd;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = a < P->nd ? (int)(grid->shape[a] + 2LL * P->nb) : 1;
        d.phys[a] = a < P->nd ? (int)grid->shape[a] : 1;
    }
    d.nb = P->nb;
    int align = pitch_align();
    long long pitch = round_up(d.n[P->nd - 1], align);
    if (P->nd == 2) {
        d.st[1] = 1;
        d.st[0] = pitch;
        d.st[2] = 0;
        d.total = (long long)d.n[0] * pitch;
    } else {
        d.st[2] = 1;
        d.st[1] = pitch;
        d.st[0] = (long long)d.n[1] * pitch;
        d.total = (long long)d.n[0] * d.st[0];
    }
    // kernels address a 2D field, or one 3D plane, with 32-bit byte offsets
    const long long span = P->nd == 2 ? d.total : d.st[0];
    if (span * 4 > 0x7fffffffLL) {
        const char* what = P->nd == 2 ? "2D field" : "3D plane";
        delete P;
        return fail(STRIDE_E_INVALID_ARG, "%s exceeds 2 GiB", what);
    }

    double c[kMaxR + 1] = {0};
    fd_weights(grid->space_order, c);
    P->nyquist = c[0];
    for (int j = 1; j <= P->R; ++j)
        P->nyquist += 2.0 * c[j] * ((j % 2) ? -1.0 : 1.0);
    P->nyquist = -P->nyquist;
    double c0 = 0;
    P->cellvol = 1.0;
    std::memset(&P->cf, 0, sizeof(P->cf));
    for (int a = 0; a < P->nd; ++a) {
        double inv = 1.0 / (grid->spacing[a] * grid->spacing[a]);
        c0 += c[0] * inv;
        for (int j = 1; j <= P->R; ++j)
            P->cf.c[a][j] = (float)(c[j] * inv);
        P->cellvol *= grid->spacing[a];
    }
    P->cf.c0 = (float)c0;
    std::memset(&P->fd1, 0, sizeof(P->fd1));
    fd1_weights(grid->space_order, P->fd1.d);
    P->fd1.r = P->R;
    for (int a = 0; a < P->nd; ++a) {
        P->fd1.inv_dx[a] = 1.0 / grid->spacing[a];
        for (int j = 1; j <= P->R; ++j)
            P->cf.d[a][j] = (float)(P->fd1.d[j] * P->fd1.inv_dx[a]);
    }
    std::memset(&P->sp, 0, sizeof(P->sp));
    if (P->nb > 0 && grid->sponge_vref > 0)
        for (int a = 0; a < P->nd; ++a) {
            double emax = 3.0 * grid->sponge_vref * std::log(1000.0) / ((double)P->nb * grid->spacing[a]);
            P->sp.e[a] = (float)(emax / ((double)P->nb * P->nb));
        }
    P->sp.half_dt = (float)(0.5 * grid->dt);
    P->boundary = grid->boundary;
    std::memset(P->pml_c0, 0, sizeof(P->pml_c0));
    std::memset(P->pml_zmax, 0, sizeof(P->pml_zmax));
    if (P->boundary == 1) {
        // the layer holds the PML instead of the sponge: the step runs undamped
        // and the layer correction adds the stretched-coordinate terms
        for (int a = 0; a < 3; ++a)
            P->sp.e[a] = 0.f;
        for (int a = 0; a < P->nd; ++a) {
            P->pml_c0[a] = (float)(c[0] / (grid->spacing[a] * grid->spacing[a]));
            if (P->nb > 0 && grid->sponge_vref > 0)
                P->pml_zmax[a] = (float)(3.0 * grid->sponge_vref * std::log(1000.0) /
                                         (2.0 * (double)P->nb * grid->spacing[a]));
        }
    }

    int ryf, wf, rya, wa, ryv, wv;
    tile_shape(P->nd, false, &ryf, &wf);
    tile_shape(P->nd, true, &rya, &wa);
    tile_shape_v(P->nd, &ryv, &wv);
    P->ls_fwd = make_shape(d, default_zc(d, false), ryf, wf);
    P->ls_adj = make_shape(d, default_zc(d, true), rya, wa);
    P->ls_adjv = make_shape(d, default_zc(d, true), ryv, wv);


    TapSet st, rt;
    if ((rc = make_taps(*P, src_xyz, nsrc, st, "source")) ||
        (rc = make_taps(*P, rec_xyz, nrec, rt, "receiver"))) {
        delete P;
        return rc;
    }
    HostTiles tsf = build_tiles(*P, st, 1.0 / P->cellvol, P->ls_fwd);
    HostTiles tsa = build_tiles(*P, st, 1.0 / P->cellvol, P->ls_adj);
    HostTiles tra = build_tiles(*P, rt, 1.0, P->ls_adj);
    HostTiles trv = build_tiles(*P, rt, 1.0, P->ls_adjv);
    std::vector<long long> ridx, sidx;
    std::vector<float> rw, sw;
    flatten_sample(rt, 1.0, ridx, rw);
    flatten_sample(st, 1.0 / P->cellvol, sidx, sw);

    // one device blob of 256-byte aligned parts: sampling taps and injection tables
    auto bytes_of = [](size_t n, size_t sz) { return (size_t)round_up((long long)(n * sz), 256); };
    size_t off = 0;
    std::vector<std::pair<size_t, std::pair<const void*, size_t>>> parts;
    auto add = [&](const void* src, size_t n, size_t sz) {
        size_t o = off;
        parts.push_back({o, {src, n * sz}});
        off += bytes_of(std::max<size_t>(n, 1), sz);
        return o;
    };
    size_t o_ridx = add(ridx.data(), ridx.size(), 8);
    size_t o_rw = add(rw.data(), rw.size(), 4);
    size_t o_sidx = add(sidx.data(), sidx.size(), 8);
    size_t o_sw = add(sw.data(), sw.size(), 4);
    size_t o_tsf_ptr = add(tsf.ptr.data(), tsf.ptr.size(), 4);
    size_t o_tsf_ent = add(tsf.ent.data(), tsf.ent.size(), sizeof(TileEntry));
    size_t o_tsa_ptr = add(tsa.ptr.data(), tsa.ptr.size(), 4);
    size_t o_tsa_ent = add(tsa.ent.data(), tsa.ent.size(), sizeof(TileEntry));
    size_t o_tra_ptr = add(tra.ptr.data(), tra.ptr.size(), 4);
    size_t o_tra_ent = add(tra.ent.data(), tra.ent.size(), sizeof(TileEntry));
    size_t o_trv_ptr = add(trv.ptr.data(), trv.ptr.size(), 4);
    size_t o_trv_ent = add(trv.ent.data(), trv.ent.size(), sizeof(TileEntry));
    std::vector<int> none(
        (size_t)std::max({P->ls_fwd.tile_blocks, P->ls_adj.tile_blocks, P->ls_adjv.tile_blocks}) + 1,
        0);
    size_t o_none = add(none.data(), none.size(), 4);
    std::vector<char> host(off, 0);
    for (auto& pt : parts)
        if (pt.second.second)
            std::memcpy(host.data() + pt.first, pt.second.first, pt.second.second);
    hipError_t e = hipGetDevice(&P->device);
    if (e == hipSuccess)
        e = hipMalloc(&P->blob, off);
    if (e == hipSuccess)
        e = hipMemcpy(P->blob, host.data(), off, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (P->blob)
            (void)hipFree(P->blob);
        delete P;
        return fail(STRIDE_E_HIP, "plan tables: %s", hipGetErrorString(e));
    }
    char* B = (char*)P->blob;
    P->src_inj = InjTable{(const int*)(B + o_tsf_ptr), (const TileEntry*)(B + o_tsf_ent)};
    P->src_img = InjTable{(const int*)(B + o_tsa_ptr), (const TileEntry*)(B + o_tsa_ent)};
    P->rec_inj = InjTable{(const int*)(B + o_tra_ptr), (const TileEntry*)(B + o_tra_ent)};
    P->rec_inj_v = InjTable{(const int*)(B + o_trv_ptr), (const TileEntry*)(B + o_trv_ent)};
    P->no_inj = InjTable{(const int*)(B + o_none), (const TileEntry*)(B + o_tra_ent)};

    P->rec_idx = (const long long*)(B + o_ridx);
    P->rec_w = (const float*)(B + o_rw);
    P->src_idx = (const long long*)(B + o_sidx);
    P->src_w = (const float*)(B + o_sw);
    *out = P;
    return STRIDE_OK;
}

int stride_plan_destroy(stride_plan_t* plan)
{
    if (!plan)
        return STRIDE_OK;
    if (plan->blob) {
        hipError_t e = hipFree(plan->blob);
        delete plan;
        if (e != hipSuccess)
            return fail(STRIDE_E_HIP, "hipFree: %s", hipGetErrorString(e));
        return STRIDE_OK;
    }
    delete plan;
    return STRIDE_OK;
}

int stride_plan_padded_shape(const stride_plan_t* plan, int64_t out[3])
{
    if (!plan || !out)
        return fail(STRIDE_E_INVALID_ARG, "NULL argument");
    for (int a = 0; a < 3; ++a)
        out[a] = plan->dims.n[a];
    return STRIDE_OK;
}

int stride_workspace_bytes(const stride_plan_t* plan, int32_t mode, size_t budget_bytes,
                           size_t* out_bytes)
{
    if (!plan || !out_bytes)
        return fail(STRIDE_E_INVALID_ARG, "NULL argument");
    Layout L = layout_of(*plan);
    if (mode == STRIDE_MODE_FORWARD) {
        *out_bytes = L.fixed_fwd;
        return STRIDE_OK;
    }
    if (mode == STRIDE_MODE_FORWARD_MEDIUM || mode == STRIDE_MODE_GRADIENT_MEDIUM) {
        if (plan->torder != 2)
            return fail(STRIDE_E_INVALID_ARG, "medium forward solves need time_order 2");
        if (plan->boundary == 1)
            return fail(STRIDE_E_INVALID_ARG, "medium forward solves use the sponge, not the PML");
        if (mode == STRIDE_MODE_FORWARD_MEDIUM || budget_bytes == 0 || budget_bytes >= L.grad_medium) {
            *out_bytes = mode == STRIDE_MODE_GRADIENT_MEDIUM ? L.grad_medium : L.medium;
            return STRIDE_OK;
        }
        // checkpointed medium gradient within the budget (steps never in place)
        if (budget_bytes < L.grad_medium_fixed + 5 * L.field)
            return fail(STRIDE_E_WORKSPACE, "budget %zu below the medium gradient minimum %zu",
                        budget_bytes, L.grad_medium_fixed + 5 * L.field);
        const long long cap = (long long)((budget_bytes - L.grad_medium_fixed) / L.field);
        const int sn = snaps_for_fields(plan->nt, cap - 1);
        if (sn < 0)
            return fail(STRIDE_E_WORKSPACE, "budget too small for checkpointing");
        const long long nf = std::max<long long>(cached_schedule(plan->nt, sn)->stats.peak_fields + 1, 5);
        *out_bytes = std::min(L.grad_medium, L.grad_medium_fixed + (size_t)nf * L.field);
        return STRIDE_OK;
    }
    if (mode != STRIDE_MODE_GRADIENT)
        return fail(STRIDE_E_INVALID_ARG,
                    "mode must be FORWARD, GRADIENT, FORWARD_MEDIUM or GRADIENT_MEDIUM");
    if (plan->boundary == 1)
        return fail(STRIDE_E_INVALID_ARG, "the PML is offered for forward solves only");
    long long nfields;
    if (budget_bytes == 0) {
        nfields = cached_schedule(plan->nt, plan->nt)->stats.peak_fields;
    } else {
        if (budget_bytes < L.fixed_grad + 4 * L.field)
            return fail(STRIDE_E_WORKSPACE, "budget %zu below the gradient minimum %zu", budget_bytes,
                        L.fixed_grad + 4 * L.field);
        long long cap = (long long)((budget_bytes - L.fixed_grad) / L.field);
        int s = snaps_for_fields(plan->nt, cap);
        if (s < 0)
            return fail(STRIDE_E_WORKSPACE, "budget too small for checkpointing");
        nfields = cached_schedule(plan->nt, s)->stats.peak_fields;
    }
    // never below the pool a gradient solve accepts (a very short schedule
    // can peak under it)
    nfields = std::max<long long>(nfields, 4);
    *out_bytes = L.fixed_grad + (size_t)nfields * L.field;
    return STRIDE_OK;
}

int stride_plan_forward(const stride_plan_t* plan, const float* vp, const float* wavelet,
                        float* traces, void* ws, size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_plan_forward");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    return forward_solve(*plan, vp, wavelet, traces, ws, ws_bytes, as_stream(stream));
}

int stride_plan_forward_static(const stride_plan_t* plan, const float* vp, const float* wavelet,
                               float* traces, void* stream)
{
    TraceRange range_("stride_plan_forward_static");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    const size_t need = layout_of(*plan).fixed_fwd;
    if (need > (size_t)STRIDE_STATIC_WORKSPACE_BYTES)
        return fail(STRIDE_E_WORKSPACE,
                    "the forward solve needs %zu bytes of workspace, beyond the static workspace "
                    "of %zu bytes (use stride_plan_forward with a caller workspace)",
                    need, (size_t)STRIDE_STATIC_WORKSPACE_BYTES);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device)
        return fail(STRIDE_E_INVALID_ARG, "the plan belongs to device %d, the current device is %d",
                    plan->device, dev);
    void* ws = nullptr;
    int rc = static_workspace(&ws);
    if (rc)
        return rc;
    return forward_solve(*plan, vp, wavelet, traces, ws, (size_t)STRIDE_STATIC_WORKSPACE_BYTES,
                         as_stream(stream));
}

int stride_plan_forward_medium(const stride_plan_t* plan, const float* vp, const float* rho,
                               const float* alpha0, int32_t att_power, const float* wavelet,
                               float* traces, void* ws, size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_plan_forward_medium");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    return forward_medium(*plan, vp, rho, alpha0, att_power, wavelet, traces, ws, ws_bytes,
                          as_stream(stream));
}

int stride_plan_gradient_medium(const stride_plan_t* plan, const float* vp, const float* rho,
                                const float* alpha0, int32_t att_power, const float* wavelet,
                                const float* observed, float* traces, double* misfit, float* dvp,
                                void* ws, size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_plan_gradient_medium");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    return gradient_medium(*plan, vp, rho, alpha0, att_power, wavelet, observed, traces, misfit, dvp,
                           ws, ws_bytes, as_stream(stream));
}

int stride_descent_step(float* vp, const float* grad, const float* mask, int64_t n, float step_size,
                        float vmin, float vmax, uint32_t* work, void* stream)
{
    g_err.clear();
    if (n < 0 || (n > 0 && (!vp || !grad || !work)))
        return fail(STRIDE_E_INVALID_ARG, "vp, grad and work must be device pointers");
    if (!(step_size >= 0.f) || !(vmin <= vmax))
        return fail(STRIDE_E_INVALID_ARG, "step_size must be >= 0 and vmin <= vmax");
    if (n == 0)
        return STRIDE_OK;
    launch_descent(vp, grad, mask, n, step_size, vmin, vmax, work, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return STRIDE_OK;
}

int stride_lowpass(const float* in, float* out, int32_t count, int32_t nt, double dt,
                   double f_max, void* stream)
{
    g_err.clear();
    if (count < 0 || nt < 1 || (count > 0 && (!in || !out)))
        return fail(STRIDE_E_INVALID_ARG, "bad low-pass arguments");
    if (!(dt > 0) || !(f_max > 0) || !(f_max * dt < 0.5))
        return fail(STRIDE_E_INVALID_ARG, "f_max must lie in (0, 1/(2 dt)) (got %g at dt %g)", f_max,
                    dt);
    const long long lds = 4LL * (2LL * lowpass_taps(dt, f_max) + 1 + nt);
    if (lds > 60 * 1024)
        return fail(STRIDE_E_INVALID_ARG,
                    "low-pass row too long: nt + 2 ceil(2/(f_max dt)) + 1 must stay within 15360");
    if (count == 0)
        return STRIDE_OK;
    launch_lowpass(in, out, count, nt, dt, f_max, as_stream(stream));
    HIP_TRY(hipGetLastError());
    return STRIDE_OK;
}

int stride_forward_save(const stride_plan_t* plan, const float* vp, const float* wavelet,
                        float* traces, void* ws, size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_forward_save");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    GradWs W;
    hipStream_t s = as_stream(stream);
    int rc = forward_save(*plan, vp, wavelet, traces, ws, ws_bytes, s, W);
    if (rc)
        return rc;
    return check_finite(finite_flag(ws), s,
                        {{traces ? traces : W.traces, nullptr, (long long)plan->nrec * plan->nt, "traces"}});
}

int stride_backward(const stride_plan_t* plan, const float* vp, const float* wavelet,
                    const float* grad_traces, float* dvp, float* dwavelet, void* ws,
                    size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_backward");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    hipStream_t s = as_stream(stream);
    int rc = backward(*plan, vp, wavelet, grad_traces, dvp, dwavelet, ws, ws_bytes, s);
    if (rc)
        return rc;
    return check_finite(finite_flag(ws), s,
                        {{dvp, nullptr, phys_points(*plan), "dvp"},
                         {dwavelet, nullptr, dwavelet ? (long long)plan->nsrc * plan->nt : 0, "dwavelet"}});
}

int stride_plan_gradient(const stride_plan_t* plan, const float* vp, const float* wavelet,
                         const float* observed, float* traces, double* misfit, float* dvp,
                         void* ws, size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_plan_gradient");
    g_err.clear();
    if (!plan)
        return fail(STRIDE_E_INVALID_ARG, "plan is NULL");
    if ((!observed && plan->nrec > 0) || !misfit || !dvp)
        return fail(STRIDE_E_INVALID_ARG, "observed, misfit and dvp must be device pointers");
    hipStream_t s = as_stream(stream);
    GradWs W;
    int rc = forward_save(*plan, vp, wavelet, traces, ws, ws_bytes, s, W);
    if (rc)
        return rc;
    launch_residual_misfit(W.traces, observed, W.residual, (long long)plan->nrec * plan->nt, misfit,
                           W.partial, s);
    rc = backward(*plan, vp, wavelet, W.residual, dvp, nullptr, ws, ws_bytes, s);
    if (rc)
        return rc;
    return check_finite(finite_flag(ws), s,
                        {{W.traces, nullptr, (long long)plan->nrec * plan->nt, "traces"},
                         {nullptr, misfit, 1, "misfit"},
                         {dvp, nullptr, phys_points(*plan), "dvp"}});
}

int stride_workspace_query(const stride_grid_t* grid, int32_t nsrc, int32_t nrec, int32_t mode,
                           size_t budget_bytes, size_t* out_bytes)
{
    g_err.clear();
    int rc = validate_grid(grid);
    if (rc)
        return rc;
    if (!out_bytes || nsrc < 0 || nrec < 0)
        return fail(STRIDE_E_INVALID_ARG, "bad arguments");
    // the tables do not change the workspace: a geometry-free plan suffices
    stride_plan P{};
    geometry_free_plan(grid, nrec, P);
    return stride_workspace_bytes(&P, mode, budget_bytes, out_bytes);
}

int stride_forward(const stride_grid_t* grid, const float* vp, const float* wavelet, int32_t nsrc,
                   const double* src_xyz, int32_t nrec, const double* rec_xyz, float* traces,
                   void* ws, size_t ws_bytes, void* stream)
{
    TraceRange range_("stride_forward");
    stride_plan_t* plan = nullptr;
    int rc = stride_plan_create(grid, nsrc, src_xyz, nrec, rec_xyz, &plan);
    if (rc)
        return rc;
    rc = stride_plan_forward(plan, vp, wavelet, traces, ws, ws_bytes, stream);
    std::string err = g_err;
    hipError_t e = hipStreamSynchronize(as_stream(stream));
    stride_plan_destroy(plan);
    g_err = err;
    if (!rc && e != hipSuccess)
        rc = fail(STRIDE_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return rc;
}

int stride_gradient(const stride_grid_t* grid, const float* vp, const float* wavelet,
                    int32_t nsrc, const double* src_xyz, int32_t nrec, const double* rec_xyz,
                    const float* observed, double* misfit, float* dvp, void* ws, size_t ws_bytes,
                    void* stream)
{
    TraceRange range_("stride_gradient");
    stride_plan_t* plan = nullptr;
    int rc = stride_plan_create(grid, nsrc, src_xyz, nrec, rec_xyz, &plan);
    if (rc)
        return rc;
    rc = stride_plan_gradient(plan, vp, wavelet, observed, nullptr, misfit, dvp, ws, ws_bytes, stream);
    std::string err = g_err;
    hipError_t e = hipStreamSynchronize(as_stream(stream));
    stride_plan_destroy(plan);
    g_err = err;
    if (!rc && e != hipSuccess)
        rc = fail(STRIDE_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return rc;
}

int stride_check_finite(int32_t on)
{
    g_check_finite = on != 0;
    return STRIDE_OK;
}

int stride_timing_enable(int32_t on)
{
    g_timer.on = on != 0;
    return STRIDE_OK;
}

int stride_timing_read(double* fwd_ms, int64_t* fwd_steps, int64_t* fwd_launches, double* adj_ms,
                       int64_t* adj_steps, int64_t* adj_launches)
{
    double t[3] = {0, 0, 0};
    long long n[3] = {0, 0, 0}, l[3] = {0, 0, 0};
    for (auto& r : g_timer.recs) {
        HIP_TRY(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
        t[r.kind] += ms;
        n[r.kind] += r.steps;
        l[r.kind] += r.launches;
        g_timer.spare.push_back(r.a);
        g_timer.spare.push_back(r.b);
    }
    g_timer.recs.clear();
    // recomputation (kind 2) runs inside the adjoint loop (kind 1): report it
    // with the forward steps and take it out of the adjoint time
    if (fwd_ms)
        *fwd_ms = t[0] + t[2];
    if (fwd_steps)
        *fwd_steps = n[0] + n[2];
    if (fwd_launches)
        *fwd_launches = l[0] + l[2];
    if (adj_ms)
        *adj_ms = t[1] - t[2];
    if (adj_steps)
        *adj_steps = n[1];
    if (adj_launches)
        *adj_launches = l[1];
    return STRIDE_OK;
}

int stride_gradient_path(const stride_grid_t* grid, int32_t nrec, size_t ws_bytes, int32_t* path,
                         int64_t* forward_steps, int32_t* segments)
{
    g_err.clear();
    int rc = validate_grid(grid);
    if (rc)
        return rc;
    if (nrec < 0)
        return fail(STRIDE_E_INVALID_ARG, "nrec must be >= 0");
    if (grid->boundary == 1)
        return fail(STRIDE_E_INVALID_ARG, "the PML is offered for forward solves only");
    stride_plan P{};
    geometry_free_plan(grid, nrec, P);
    Layout L = layout_of(P);
    if (ws_bytes < L.fixed_grad + 4 * L.field)
        return fail(STRIDE_E_WORKSPACE, "gradient workspace needs at least %zu bytes (got %zu)",
                    L.fixed_grad + 4 * L.field, ws_bytes);
    const long long nfields = (long long)((ws_bytes - L.fixed_grad) / L.field);
    const int sn = snaps_for_fields(P.nt, nfields);
    if (sn < 0)
        return fail(STRIDE_E_WORKSPACE, "workspace too small for checkpointing");
    GradPath g = grad_path(P, nfields, sn);
    if (path)
        *path = g.kind;
    if (forward_steps)
        *forward_steps = g.forward_steps;
    if (segments)
        *segments = g.kind == GradPath::kSegmented ? (int32_t)g.starts.size() : 0;
    return STRIDE_OK;
}

int stride_schedule_info(int32_t nt, int64_t fields, int32_t* snaps, int64_t* forward_steps,
                         int32_t* peak_fields)
{
    if (nt < 1)
        return fail(STRIDE_E_INVALID_ARG, "nt must be >= 1");
    int s = snaps_for_fields(nt, fields);
    if (s < 0)
        return fail(STRIDE_E_WORKSPACE, "%lld wavefields cannot hold the checkpointing schedule",
                    (long long)fields);
    ScheduleStats st = cached_schedule(nt, s)->stats;
    if (snaps)
        *snaps = s;
    if (forward_steps)
        *forward_steps = st.forward_steps;
    if (peak_fields)
        *peak_fields = st.peak_fields;
    return STRIDE_OK;
}

}  // extern "C"
