// Continuous-batching engine: many shots on one padded grid advance together,
// one time step per tick, in shared batched launches.
//
// The paper parallelises over shots, each worker computing one shot gradient
// at a time and keeping its objects warm on its node or accelerator
// (Sec. 2.5; Sec. 3.3 dispatches all shots at once and workers start as soon
// as work arrives).  On one GPU the same shot parallelism becomes batching:
// each slot of the engine holds one shot (forward solve or checkpointed
// gradient) with its own model, geometry, dt and time index; a tick advances
// every active slot by one forward or one adjoint step, in one batched launch
// per direction.  Slots join and leave at chunk boundaries, so new work is
// admitted while other shots are in flight.
//
// Per chunk the host writes each slot's step parameters for every tick into a
// pinned staging table (double-buffered; active entries packed from row 0 so
// launches cover only occupied rows), copies it to the device, and replays a
// hipGraph of the chunk's launches (captured once per chunk length and launch
// heights).  Chunks have a fixed length; a slot whose phase ends inside one
// idles to its end.  Phase transitions run as ordinary launches at chunk
// boundaries: the last trace sample, the residual and misfit, and the
// gradient finalise.  A shot's arithmetic is the single-shot kernels' body,
// so its result is the same bits alone and in any batch.
#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "plan.h"

using namespace stride;

namespace {

// Launch groups of a tick, one batched launch each (empty groups launch
// nothing).  Stage-0 groups run first; the fourth-order corrections read the
// p / q fields that kPrep rows of the same tick wrote.
enum Group {
    kGFwd = 0,       // forward leapfrog step
    kGFwdV,          // forward step storing v = L u + S (full history, second order)
    kGPrep,          // k (L A + St): fourth-order forward p, adjoint p and q
    kGAdj,           // adjoint step with the fused imaging (checkpointed, second order)
    kGAdjImage,      // adjoint step adding two imaging terms from v (full history)
    kGAdjPlain,      // adjoint step without imaging (full history)
    kGFwdCorrect,    // fourth-order forward correction (stage 1)
    kGAdjCorrect,    // fourth-order adjoint correction with imaging (stage 1)
    kGroups
};
constexpr bool kGroupAdjoint[kGroups] = {false, false, false, true, true, true, false, true};
constexpr int kGroupMode[kGroups] = {kStep, kStepV, kPrep, kStep, kImageV, kAdjPlain, kCorrect, kCorrect};

// A fourth-order adjoint step has two kPrep rows (p and q); every other
// group has at most one row per slot.
int group_rows(int g, int max_slots) { return g == kGPrep ? 2 * max_slots : max_slots; }

struct SlotJob {
    bool used = false;
    bool finished = false;
    const stride_plan* P = nullptr;
    int mode = STRIDE_MODE_FORWARD;
    const float* vp = nullptr;
    const float* wavelet = nullptr;
    const float* observed = nullptr;
    float* traces = nullptr;
    double* misfit = nullptr;
    float* dvp = nullptr;
    FwdWs F{};
    int cur = 0, n = 0;                  // forward sweeps: ping-pong index and time index
    GradWs W;
    std::unique_ptr<StepCursor> cursor;  // checkpointed gradient
    bool history = false;                // gradient keeping v^n (second order) or p^n (fourth)
    int phase = 0;                       // gradient: 0 forward sweep, 1 recompute + adjoint
    int m = 0;                           // full-history / segmented adjoint: next step
    int wa = 0;                          // adjoint ping-pong
    long long left = 0;                  // ticks until the current phase ends
    // segmented history: segment starts, v buffer pool[0, vbuf), working pair
    // pool[vbuf], pool[vbuf + 1], start state of segment k in pool[vbuf + 2k],
    // pool[vbuf + 2k + 1]; fc / fp hold u^n / u^{n-1} of the sweep in progress
    bool seg = false;
    GradPath path;
    int sk = 0;                          // phase 1: segment in progress
    bool recompute = false;              // phase 1: recomputing segment sk's v
    int rn = 0;                          // recompute: next step
    float* fc = nullptr;
    float* fp = nullptr;
};

bool same_layout(const Dims& a, const Dims& b)
{
    if (a.nd != b.nd || a.nb != b.nb || a.total != b.total)
        return false;
    for (int i = 0; i < 3; ++i)
        if (a.n[i] != b.n[i] || a.st[i] != b.st[i] || a.phys[i] != b.phys[i])
            return false;
    return true;
}

}  // namespace

struct stride_engine {
    Dims dims;
    int R;
    StencilCoef cf;
    LaunchShape ls_fwd, ls_adj;
    LaunchShape ls_adjv;      // adjoint steps imaging from a stored v (the single-shot shape)
    int max_slots, max_samples, tmax;
    int ntap;                 // taps per receiver of the engine's grid (linear or sinc)
    bool graphs;
    stride_plan_t* shape_plan = nullptr;   // geometry-free plan fixing the layout
    std::vector<SlotJob> slots;
    int group_off[kGroups + 1] = {};        // row offset of each group within a tick
    SlotStep* d_table = nullptr;           // [tmax][rows per tick] on the device
    SlotStep* h_stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_i = 0;
    std::map<std::array<int, kGroups + 1>, hipGraphExec_t> execs;   // (ticks, launch heights)
    long long ticks_total = 0;

    int tick_rows() const { return group_off[kGroups]; }
};

namespace {

// Rows of one slot for one tick, appended to the groups' row lists.
struct TickRows {
    SlotStep* row[kGroups];
    int count[kGroups];
    void add(int g, const SlotStep& t) { row[g][count[g]++] = t; }
};

SlotStep make_row(const stride_plan& P, const StepParams& p)
{
    SlotStep t{};
    t.p = p;
    t.sp = P.sp;
    t.active = 1;
    return t;
}

// Forward step n from u^n = A to u^{n+1} = C (B = u^{n-1}, overwritten by C),
// sampling `smp`; fourth order: p = k (L u^n + St^n) into `pbuf`, then the
// correction.  With `keep` set (full history) the step also stores v^n (second
// order) or writes p^n to `keep` instead of `pbuf` (fourth order).
void forward_rows(const stride_plan& P, TickRows& R, const float* A, const float* B, float* C,
                  const float* K, int n, const float* wavelet, SampleSet smp, float* pbuf,
                  float* keep)
{
    StepParams p = base_params(P);
    p.K = K;
    p.step = n;
    if (P.torder == 2) {
        p.A = A;
        p.B = B;
        p.C = C;
        p.inj_sig = wavelet;
        p.smp = smp;
        if (keep)
            p.V = keep;
        R.add(keep ? kGFwdV : kGFwd, make_row(P, p));
        return;
    }
    float* pp = keep ? keep : pbuf;
    p.A = A;
    p.C = pp;
    p.inj_sig = wavelet;
    p.smp = smp;
    R.add(kGPrep, make_row(P, p));
    StepParams q = base_params(P);
    q.A = pp;
    q.D = A;
    q.B = B;
    q.C = C;
    q.K = K;
    q.step = n;
    R.add(kGFwdCorrect, make_row(P, q));
}

// Adjoint step m imaging from v^m = V[m - j] (pairs as on the full-history
// path; V2 only inside [j, e)).
void adjoint_v_row(const stride_plan& P, TickRows& R, SlotJob& J, int m, int j, int e)
{
    StepParams c = base_params(P);
    c.A = J.W.w[J.wa];
    c.B = J.W.w[1 - J.wa];
    c.C = J.W.w[1 - J.wa];
    c.K = J.W.k;
    c.G = J.W.G;
    c.step = m;
    c.inj = P.rec_inj_v;
    c.inj_sig = J.W.residual;
    c.inj_stride = P.nt;
    c.img = P.no_inj;
    c.V = J.W.pool[m - j];
    c.V2 = m + 1 < e ? J.W.pool[m + 1 - j] : nullptr;
    R.add(m % 2 == 0 ? kGAdjImage : kGAdjPlain, make_row(P, c));
    J.wa = 1 - J.wa;
}

// Adjoint step m of a gradient whose imaging operand is kept in
// pool[m - j] (m in [j, e)): v^m (second order, above) or p^m (fourth order:
// q = k L w^{m+1}, then the correction with p^m, two rows).
void adjoint_hist_row(const stride_plan& P, TickRows& R, SlotJob& J, int m, int j, int e)
{
    if (P.torder == 2) {
        adjoint_v_row(P, R, J, m, j, e);
        return;
    }
    StepParams q = base_params(P);
    q.A = J.W.w[J.wa];
    q.C = J.W.q;
    q.K = J.W.k;
    q.step = m;
    q.inj = P.no_inj;
    R.add(kGPrep, make_row(P, q));
    StepParams c = base_params(P);
    c.A = J.W.q;
    c.U = J.W.pool[m - j];
    c.D = J.W.w[J.wa];
    c.B = J.W.w[1 - J.wa];
    c.C = J.W.w[1 - J.wa];
    c.K = J.W.k;
    c.G = J.W.G;
    c.step = m;
    c.inj = P.rec_inj;
    c.inj_sig = J.W.residual;
    c.inj_stride = P.nt;
    c.img = P.no_inj;
    R.add(kGAdjCorrect, make_row(P, c));
    J.wa = 1 - J.wa;
}

int fill_seg(SlotJob& J, TickRows& R)
{
    const stride_plan& P = *J.P;
    const std::vector<int>& st = J.path.starts;
    const int K = (int)st.size(), last = st[K - 1];
    if (J.phase == 0) {
        const int n = J.n;
        float* C = seg_sweep_out(J.path, J.W.pool, J.W.w, J.fc, J.fp, n + 1);
        forward_rows(P, R, J.fc, J.fp, C, J.W.k, n, J.wavelet, rec_samples(P, J.W.traces), J.W.p,
                     n >= last ? J.W.pool[n - last] : nullptr);
        J.fp = J.fc;
        J.fc = C;
        ++J.n;
        return STRIDE_OK;
    }
    const int j = st[J.sk], e = J.sk + 1 < K ? st[J.sk + 1] : P.nt;
    if (J.recompute) {
        // v^n (p^n) of segment sk from its start state, u in place
        const int n = J.rn++;
        forward_rows(P, R, J.fc, J.fp, J.fp, J.W.k, n, J.wavelet, SampleSet{}, J.W.p,
                     J.W.pool[n - j]);
        std::swap(J.fc, J.fp);
        if (J.rn == e) {
            J.recompute = false;
            J.m = e - 1;
        }
        return STRIDE_OK;
    }
    const int m = J.m--;
    adjoint_hist_row(P, R, J, m, j, e);
    if (m == j && J.sk > 0) {
        // next: segment sk - 1, recomputed from its start state (x_0 = 0 in
        // the zeroed working pair for the first segment)
        const int k = --J.sk;
        J.recompute = true;
        J.rn = st[k];
        J.fc = J.W.pool[J.path.vbuf + 2 * k];
        J.fp = J.W.pool[J.path.vbuf + 2 * k + 1];
    }
    return STRIDE_OK;
}

int fill_tick(SlotJob& J, TickRows& R)
{
    const stride_plan& P = *J.P;
    if (J.seg)
        return fill_seg(J, R);
    if (J.mode == STRIDE_MODE_FORWARD) {
        forward_rows(P, R, J.F.u[J.cur], J.F.u[1 - J.cur], J.F.u[1 - J.cur], J.F.k, J.n, J.wavelet,
                     rec_samples(P, J.traces), J.F.p, nullptr);
        J.cur = 1 - J.cur;
        ++J.n;
        return STRIDE_OK;
    }
    if (J.history) {
        // full history: u rotates in the adjoint fields during the forward sweep
        if (J.phase == 0) {
            float* u[2] = {J.W.w[0], J.W.w[1]};
            forward_rows(P, R, u[J.cur], u[1 - J.cur], u[1 - J.cur], J.W.k, J.n, J.wavelet,
                         rec_samples(P, J.W.traces), nullptr, J.W.pool[J.n]);
            J.cur = 1 - J.cur;
            ++J.n;
            return STRIDE_OK;
        }
        // imaging terms in pairs (second order), or q and the correction
        // with p^m kept (fourth order)
        adjoint_hist_row(P, R, J, J.m--, 0, P.nt);
        return STRIDE_OK;
    }
    StepOp op;
    if (!J.cursor->next(op))
        return fail(STRIDE_E_WORKSPACE, "checkpoint schedule ended early (pool overflow)");
    if (!op.reverse) {
        forward_rows(P, R, J.W.pool[op.a], J.W.pool[op.b], J.W.pool[op.c], J.W.k, op.step,
                     J.wavelet, op.first_sweep ? rec_samples(P, J.W.traces) : SampleSet{}, J.W.p,
                     nullptr);
        return STRIDE_OK;
    }
    StepParams c = base_params(P);
    c.B = J.W.w[1 - J.wa];
    c.C = J.W.w[1 - J.wa];
    c.K = J.W.k;
    c.G = J.W.G;
    c.step = op.step;
    c.inj = P.rec_inj;
    c.inj_sig = J.W.residual;
    c.inj_stride = P.nt;
    if (P.torder == 2) {
        c.A = J.W.w[J.wa];
        c.U = J.W.pool[op.a];
        c.img = P.src_img;
        c.img_sig = J.wavelet;
        c.img_stride = P.nt;
        R.add(kGAdj, make_row(P, c));
    } else {
        // p = k (L u^m + St^m), q = k L w^{m+1}, then w^m and the imaging
        StepParams p = base_params(P);
        p.A = J.W.pool[op.a];
        p.C = J.W.p;
        p.K = J.W.k;
        p.step = op.step;
        p.inj_sig = J.wavelet;
        R.add(kGPrep, make_row(P, p));
        StepParams q = base_params(P);
        q.A = J.W.w[J.wa];
        q.C = J.W.q;
        q.K = J.W.k;
        q.step = op.step;
        q.inj = P.no_inj;
        R.add(kGPrep, make_row(P, q));
        c.A = J.W.q;
        c.U = J.W.p;
        c.D = J.W.w[J.wa];
        c.img = P.no_inj;
        R.add(kGAdjCorrect, make_row(P, c));
    }
    J.wa = 1 - J.wa;
    return STRIDE_OK;
}

// gy[g]: rows of group g each launch covers (0 = no launch).
void launch_chunk(stride_engine* E, int ticks, const int* gy, hipStream_t s)
{
    const int sample_threads = E->max_samples * sample_lanes(E->ntap);
    for (int t = 0; t < ticks; ++t) {
        const SlotStep* base = E->d_table + (size_t)t * E->tick_rows();
        for (int g = 0; g < kGroups; ++g) {
            if (!gy[g])
                continue;
            const bool adj = kGroupAdjoint[g];
            // traces are sampled by the forward step (fourth order: its kPrep row)
            const bool smp = g == kGFwd || g == kGFwdV || g == kGPrep;
            const LaunchShape& ls = !adj                                     ? E->ls_fwd
                                    : (g == kGAdjImage || g == kGAdjPlain) ? E->ls_adjv
                                                                           : E->ls_adj;
            launch_step_batched(E->dims, E->R, adj, kGroupMode[g], E->cf, ls, base + E->group_off[g],
                                gy[g], smp ? sample_threads : 0, s);
        }
    }
}

int get_exec(stride_engine* E, int ticks, const int* gy, hipStream_t s, hipGraphExec_t* out)
{
    std::array<int, kGroups + 1> key{};
    key[0] = ticks;
    for (int g = 0; g < kGroups; ++g)
        key[g + 1] = gy[g];
    auto it = E->execs.find(key);
    if (it != E->execs.end()) {
        *out = it->second;
        return STRIDE_OK;
    }
    hipGraph_t g = nullptr;
    STRIDE_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    launch_chunk(E, ticks, gy, s);
    hipError_t e = hipStreamEndCapture(s, &g);
    if (e != hipSuccess)
        return fail(STRIDE_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess)
        return fail(STRIDE_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    E->execs[key] = x;
    *out = x;
    return STRIDE_OK;
}

// Ticks of a gradient's second phase (recomputation and adjoint).
long long second_phase_ticks(const SlotJob& J)
{
    const int nt = J.P->nt;
    if (J.seg)
        return nt + J.path.starts.back();
    return J.history ? nt : J.cursor->forward_steps() - (nt - 1) + nt;
}

// Work between phases, enqueued after the chunk that ended the phase.
void end_phase(stride_engine* E, SlotJob& J, hipStream_t s)
{
    (void)E;
    const stride_plan& P = *J.P;
    if (J.mode == STRIDE_MODE_FORWARD) {
        launch_sample(rec_samples(P, J.traces), J.F.u[J.cur], P.nt - 1, s);
        J.finished = true;
        return;
    }
    if (J.phase == 0) {
        // the forward sweep ended in x_{nt-1}: last sample, residual, misfit
        const float* last = J.seg       ? J.fc
                            : J.history ? J.W.w[J.cur]
                                        : J.W.pool[J.cursor->cur()];
        launch_sample(rec_samples(P, J.W.traces), last, P.nt - 1, s);
        launch_residual_misfit(J.W.traces, J.observed, J.W.residual, (long long)P.nrec * P.nt,
                               J.misfit, J.W.partial, s);
        if (J.traces)
            launch_copy(J.traces, J.W.traces, (long long)P.nrec * P.nt, s);
        if (J.history) {
            // v^{nt-1} (p^{nt-1}) is never formed and meets w^{nt} = 0; the
            // adjoint fields held u and start at zero
            launch_fill(J.W.pool[P.nt - 1], P.dims.total, 0.f, s);
            launch_fill(J.W.w[0], P.dims.total, 0.f, s);
            launch_fill(J.W.w[1], P.dims.total, 0.f, s);
            J.m = P.nt - 1;
            J.wa = 0;
        }
        if (J.seg) {
            // as above for the last segment's v buffer; the working pair
            // holds x_0 = 0 for the first segment's recomputation
            const int last_start = J.path.starts.back();
            launch_fill(J.W.pool[P.nt - 1 - last_start], P.dims.total, 0.f, s);
            for (float* f : {J.W.w[0], J.W.w[1], J.W.pool[J.path.vbuf], J.W.pool[J.path.vbuf + 1]})
                launch_fill(f, P.dims.total, 0.f, s);
            J.sk = (int)J.path.starts.size() - 1;
            J.recompute = false;
            J.m = P.nt - 1;
            J.wa = 0;
        }
        J.phase = 1;
        J.left = second_phase_ticks(J);
        return;
    }
    // the fourth-order accumulator holds k G
    launch_finalize_dvp(P.dims, J.W.G, P.torder == 4 ? J.W.k : nullptr, J.vp, J.dvp, J.W.w[0],
                        J.W.w[1], s);
    J.finished = true;
}

}  // namespace

extern "C" {

int stride_engine_create(const stride_grid_t* grid, int32_t max_slots, int32_t max_receivers,
                         int32_t max_chunk, int32_t use_graphs, stride_engine_t** out)
{
    if (!out || max_slots < 1 || max_slots > 4096 || max_receivers < 0 || max_chunk < 1)
        return fail(STRIDE_E_INVALID_ARG, "bad engine arguments");
    *out = nullptr;
    stride_plan_t* sp = nullptr;
    int rc = stride_plan_create(grid, 0, nullptr, 0, nullptr, &sp);
    if (rc)
        return rc;
    auto* E = new stride_engine();
    E->shape_plan = sp;
    E->dims = sp->dims;
    E->R = sp->R;
    E->cf = sp->cf;
    E->ls_fwd = sp->ls_fwd;
    E->ls_adj = sp->ls_adj;
    E->ls_adjv = sp->ls_adjv;
    E->max_slots = max_slots;
    E->max_samples = max_receivers;
    E->ntap = sp->ntap;
    int t = 1;
    while (t * 2 <= max_chunk)
        t *= 2;
    E->tmax = t;
    E->graphs = use_graphs != 0;
    E->slots.resize(max_slots);
    for (int g = 0; g < kGroups; ++g)
        E->group_off[g + 1] = E->group_off[g] + group_rows(g, max_slots);
    size_t bytes = sizeof(SlotStep) * (size_t)E->tmax * E->tick_rows();
    hipError_t e = hipMalloc((void**)&E->d_table, bytes);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc((void**)&E->h_stage[i], bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&E->stage_ev[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        stride_engine_destroy(E);
        return fail(STRIDE_E_HIP, "engine allocation: %s", hipGetErrorString(e));
    }
    *out = E;
    return STRIDE_OK;
}

int stride_engine_destroy(stride_engine_t* E)
{
    if (!E)
        return STRIDE_OK;
    (void)hipDeviceSynchronize();
    for (auto& kv : E->execs)
        (void)hipGraphExecDestroy(kv.second);
    for (int i = 0; i < 2; ++i) {
        if (E->h_stage[i])
            (void)hipHostFree(E->h_stage[i]);
        if (E->stage_ev[i])
            (void)hipEventDestroy(E->stage_ev[i]);
    }
    if (E->d_table)
        (void)hipFree(E->d_table);
    if (E->shape_plan)
        stride_plan_destroy(E->shape_plan);
    delete E;
    return STRIDE_OK;
}

int stride_engine_attach(stride_engine_t* E, const stride_plan_t* plan, int32_t mode,
                         const float* vp, float vp_max, const float* wavelet, const float* observed,
                         float* traces, double* misfit, float* dvp, void* ws, size_t ws_bytes,
                         void* stream, int32_t* slot)
{
    TraceRange range_("stride_engine_attach");
    if (!E || !plan || !slot)
        return fail(STRIDE_E_INVALID_ARG, "NULL engine, plan or slot");
    if (!same_layout(E->dims, plan->dims) || E->R != plan->R || E->ntap != plan->ntap ||
        std::memcmp(&E->cf, &plan->cf, sizeof(StencilCoef)) != 0)
        return fail(STRIDE_E_INVALID_ARG, "plan grid does not match the engine grid");
    if (plan->boundary != 0)
        return fail(STRIDE_E_INVALID_ARG, "the engine runs solves with the sponge only");
    if (plan->nrec > E->max_samples)
        return fail(STRIDE_E_INVALID_ARG, "plan has %d receivers; the engine samples at most %d",
                    plan->nrec, E->max_samples);
    if (!vp || (!wavelet && plan->nsrc > 0))
        return fail(STRIDE_E_INVALID_ARG, "vp and wavelet must be device pointers");
    int free_slot = -1;
    for (int i = 0; i < E->max_slots; ++i)
        if (!E->slots[i].used) {
            free_slot = i;
            break;
        }
    if (free_slot < 0)
        return fail(STRIDE_E_INVALID_ARG, "no free slot");
    hipStream_t s = (hipStream_t)stream;
    SlotJob J;
    J.P = plan;
    J.mode = mode;
    J.vp = vp;
    J.wavelet = wavelet;
    J.observed = observed;
    J.traces = traces;
    J.misfit = misfit;
    J.dvp = dvp;
    int rc;
    if (mode == STRIDE_MODE_FORWARD) {
        if (!traces && plan->nrec > 0)
            return fail(STRIDE_E_INVALID_ARG, "forward slots need traces");
        if ((rc = fwd_ws(*plan, ws, ws_bytes, J.F)))
            return rc;
        rc = vp_max > 0 ? check_cfl(*plan, vp_max) : check_vp(*plan, vp, J.F.flags, s);
        if (rc)
            return rc;
        launch_prep_k(plan->dims, vp, plan->g.dt, J.F.k, s);
        launch_fill(J.F.u[0], plan->dims.total, 0.f, s);
        launch_fill(J.F.u[1], plan->dims.total, 0.f, s);
        J.left = plan->nt - 1;
    } else if (mode == STRIDE_MODE_GRADIENT) {
        if ((!observed && plan->nrec > 0) || !misfit || !dvp)
            return fail(STRIDE_E_INVALID_ARG, "gradient slots need observed, misfit and dvp");
        if ((rc = grad_ws(*plan, ws, ws_bytes, J.W)))
            return rc;
        rc = vp_max > 0 ? check_cfl(*plan, vp_max) : check_vp(*plan, vp, J.W.flags, s);
        if (rc)
            return rc;
        launch_prep_k(plan->dims, vp, plan->g.dt, J.W.k, s);
        // the single-shot path for this workspace (the same bits): every
        // state fits, the forward keeps v^n (p^n) and the adjoint images from
        // it; segmented history; or the binomial schedule's own step cursor
        J.path = grad_path(*plan, (long long)J.W.pool.size(), J.W.snaps);
        J.history = J.path.kind == GradPath::kFull;
        J.seg = J.path.kind == GradPath::kSegmented;
        if (J.history || J.seg) {
            for (float* f : {J.W.G, J.W.w[0], J.W.w[1]})
                launch_fill(f, plan->dims.total, 0.f, s);
            J.fc = J.W.w[0];
            J.fp = J.W.w[1];
        } else {
            J.cursor = std::make_unique<StepCursor>(plan->nt, J.W.snaps, J.W.peak);
            for (float* f : {J.W.pool[0], J.W.pool[1], J.W.G, J.W.w[0], J.W.w[1]})
                launch_fill(f, plan->dims.total, 0.f, s);
        }
        J.phase = 0;
        J.left = plan->nt - 1;
    } else {
        return fail(STRIDE_E_INVALID_ARG, "mode must be FORWARD or GRADIENT");
    }
    STRIDE_HIP_TRY(hipGetLastError());
    J.used = true;
    E->slots[free_slot] = std::move(J);
    *slot = free_slot;
    return STRIDE_OK;
}

int stride_engine_run(stride_engine_t* E, int32_t max_ticks, void* stream, int32_t* ticks_run,
                      int32_t* finished)
{
    TraceRange range_("stride_engine_run");
    if (!E || !ticks_run)
        return fail(STRIDE_E_INVALID_ARG, "NULL engine or ticks_run");
    hipStream_t s = (hipStream_t)stream;
    *ticks_run = 0;
    if (finished)
        for (int i = 0; i < E->max_slots; ++i)
            finished[i] = 0;
    // Fixed-length chunks: a slot whose phase ends inside the chunk idles to
    // its end, so one slot's phase end does not cut the chunk for the others.
    long long cap = std::min<long long>(std::max(1, max_ticks), E->tmax);
    long long longest = 0;
    for (auto& J : E->slots)
        if (J.used && !J.finished)
            longest = std::max(longest, J.left);
    if (longest == 0)
        return STRIDE_OK;
    int ticks = 1;
    while (ticks < std::min(longest, cap))
        ticks *= 2;
    if (ticks > cap)
        ticks /= 2;

    // per-tick slot tables, each group's active rows packed from its first
    // row, in the pinned staging buffer
    int si = E->stage_i;
    if (E->stage_used[si])
        STRIDE_HIP_TRY(hipEventSynchronize(E->stage_ev[si]));
    SlotStep* H = E->h_stage[si];
    const size_t per_tick = (size_t)E->tick_rows();
    size_t bytes = sizeof(SlotStep) * (size_t)ticks * per_tick;
    int rows[kGroups] = {};
    std::vector<int> counts((size_t)ticks * kGroups, 0);
    std::vector<long long> used_ticks(E->max_slots, 0);
    for (int t = 0; t < ticks; ++t) {
        SlotStep* tick = H + (size_t)t * per_tick;
        TickRows R;
        for (int g = 0; g < kGroups; ++g) {
            R.row[g] = tick + E->group_off[g];
            R.count[g] = 0;
        }
        for (int j = 0; j < E->max_slots; ++j) {
            SlotJob& J = E->slots[j];
            if (!J.used || J.finished || used_ticks[j] >= J.left)
                continue;
            int rc = fill_tick(J, R);
            if (rc)
                return rc;
            ++used_ticks[j];
        }
        for (int g = 0; g < kGroups; ++g) {
            counts[(size_t)t * kGroups + g] = R.count[g];
            rows[g] = std::max(rows[g], R.count[g]);
        }
    }
    // round launch heights up to powers of two so that captured graphs
    // repeat; rows past a tick's count up to the height are inactive
    int gy[kGroups];
    for (int g = 0; g < kGroups; ++g) {
        int h = 0;
        if (rows[g]) {
            h = 1;
            while (h < rows[g])
                h *= 2;
            h = std::min(h, group_rows(g, E->max_slots));
        }
        gy[g] = h;
        for (int t = 0; t < ticks; ++t) {
            SlotStep* r = H + (size_t)t * per_tick + E->group_off[g];
            const int c = counts[(size_t)t * kGroups + g];
            if (h > c)
                std::memset((void*)(r + c), 0, sizeof(SlotStep) * (size_t)(h - c));
        }
    }
    STRIDE_HIP_TRY(hipMemcpyAsync(E->d_table, H, bytes, hipMemcpyHostToDevice, s));
    STRIDE_HIP_TRY(hipEventRecord(E->stage_ev[si], s));
    E->stage_used[si] = true;
    E->stage_i = 1 - si;

    if (E->graphs && s != nullptr) {
        hipGraphExec_t x = nullptr;
        int rc = get_exec(E, ticks, gy, s, &x);
        if (rc)
            return rc;
        STRIDE_HIP_TRY(hipGraphLaunch(x, s));
    } else {
        launch_chunk(E, ticks, gy, s);
    }
    for (int j = 0; j < E->max_slots; ++j) {
        SlotJob& J = E->slots[j];
        if (!J.used || J.finished)
            continue;
        J.left -= used_ticks[j];
        if (J.left == 0)
            end_phase(E, J, s);
        if (J.finished && finished)
            finished[j] = 1;
    }
    STRIDE_HIP_TRY(hipGetLastError());
    E->ticks_total += ticks;
    *ticks_run = ticks;
    return STRIDE_OK;
}

int stride_engine_detach(stride_engine_t* E, int32_t slot)
{
    if (!E || slot < 0 || slot >= E->max_slots || !E->slots[slot].used)
        return fail(STRIDE_E_INVALID_ARG, "bad slot");
    E->slots[slot] = SlotJob();
    return STRIDE_OK;
}

int stride_engine_slot_ticks(const stride_engine_t* E, int32_t slot, int64_t* ticks_left)
{
    if (!E || !ticks_left || slot < 0 || slot >= E->max_slots || !E->slots[slot].used)
        return fail(STRIDE_E_INVALID_ARG, "bad slot");
    const SlotJob& J = E->slots[slot];
    long long left = J.finished ? 0 : J.left;
    if (J.mode == STRIDE_MODE_GRADIENT && J.phase == 0 && !J.finished)
        left += second_phase_ticks(J);
    *ticks_left = left;
    return STRIDE_OK;
}

int stride_accumulate(float* dst, const float* src, int64_t n, void* stream)
{
    if (!dst || !src || n < 0)
        return fail(STRIDE_E_INVALID_ARG, "bad accumulate arguments");
    launch_accumulate(dst, src, n, (hipStream_t)stream);
    STRIDE_HIP_TRY(hipGetLastError());
    return STRIDE_OK;
}

}  // extern "C"
