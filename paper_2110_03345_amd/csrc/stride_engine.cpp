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
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "plan.h"

using namespace stride;

namespace {

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
    int cur = 0, n = 0;                  // forward mode: ping-pong index and time index
    GradWs W;
    std::unique_ptr<StepCursor> cursor;  // gradient mode
    int phase = 0;                       // gradient: 0 forward sweep, 1 recompute + adjoint
    int wa = 0;                          // adjoint ping-pong
    long long left = 0;                  // ticks until the current phase ends
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
    int max_slots, max_samples, tmax;
    int ntap;                 // taps per receiver of the engine's grid (linear or sinc)
    bool graphs;
    stride_plan_t* shape_plan = nullptr;   // geometry-free plan fixing the layout
    std::vector<SlotJob> slots;
    SlotStep* d_table = nullptr;           // [tmax][2][max_slots] on the device
    SlotStep* h_stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    bool stage_used[2] = {false, false};
    int stage_i = 0;
    std::map<long long, hipGraphExec_t> execs;   // key: (ticks, rows per launch)
    long long ticks_total = 0;
};

namespace {

int fill_tick(stride_engine* E, SlotJob& J, SlotStep* fwd, SlotStep* adj)
{
    const stride_plan& P = *J.P;
    if (J.mode == STRIDE_MODE_FORWARD) {
        SlotStep& t = *fwd;
        t.p = base_params(P);
        t.p.A = J.F.u[J.cur];
        t.p.B = J.F.u[1 - J.cur];
        t.p.C = J.F.u[1 - J.cur];
        t.p.K = J.F.k;
        t.p.step = J.n;
        t.p.inj_sig = J.wavelet;
        t.p.smp = rec_samples(P, J.traces);
        t.sp = P.sp;
        t.active = 1;
        J.cur = 1 - J.cur;
        ++J.n;
        return 1;
    }
    StepOp op;
    if (!J.cursor->next(op))
        return fail(STRIDE_E_WORKSPACE, "checkpoint schedule ended early (pool overflow)");
    if (!op.reverse) {
        SlotStep& t = *fwd;
        t.p = base_params(P);
        t.p.A = J.W.pool[op.a];
        t.p.B = J.W.pool[op.b];
        t.p.C = J.W.pool[op.c];
        t.p.K = J.W.k;
        t.p.step = op.step;
        t.p.inj_sig = J.wavelet;
        if (op.first_sweep)
            t.p.smp = rec_samples(P, J.W.traces);
        t.sp = P.sp;
        t.active = 1;
        return 1;
    }
    SlotStep& t = *adj;
    t.p = base_params(P);
    t.p.A = J.W.w[J.wa];
    t.p.B = J.W.w[1 - J.wa];
    t.p.C = J.W.w[1 - J.wa];
    t.p.K = J.W.k;
    t.p.U = J.W.pool[op.a];
    t.p.G = J.W.G;
    t.p.step = op.step;
    t.p.inj = P.rec_inj;
    t.p.inj_sig = J.W.residual;
    t.p.inj_stride = P.nt;
    t.p.img = P.src_img;
    t.p.img_sig = J.wavelet;
    t.p.img_stride = P.nt;
    t.sp = P.sp;
    t.active = 1;
    J.wa = 1 - J.wa;
    return 2;
}

// gy_fwd / gy_adj: rows of the per-tick tables each launch covers (0 = no launch).
void launch_chunk(stride_engine* E, int ticks, int gy_fwd, int gy_adj, hipStream_t s)
{
    for (int t = 0; t < ticks; ++t) {
        const SlotStep* base = E->d_table + (size_t)t * 2 * E->max_slots;
        if (gy_fwd)
            launch_step_batched(E->dims, E->R, false, E->cf, E->ls_fwd, base, gy_fwd,
                                E->max_samples * sample_lanes(E->ntap), s);
        if (gy_adj)
            launch_step_batched(E->dims, E->R, true, E->cf, E->ls_adj, base + E->max_slots, gy_adj, 0, s);
    }
}

int get_exec(stride_engine* E, int ticks, int gy_fwd, int gy_adj, hipStream_t s,
             hipGraphExec_t* out)
{
    long long key = ((long long)ticks * 8192 + gy_fwd) * 8192 + gy_adj;
    auto it = E->execs.find(key);
    if (it != E->execs.end()) {
        *out = it->second;
        return STRIDE_OK;
    }
    hipGraph_t g = nullptr;
    STRIDE_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    launch_chunk(E, ticks, gy_fwd, gy_adj, s);
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

// Work between phases, enqueued after the chunk that ended the phase.
void end_phase(stride_engine* E, SlotJob& J, hipStream_t s)
{
    const stride_plan& P = *J.P;
    if (J.mode == STRIDE_MODE_FORWARD) {
        launch_sample(rec_samples(P, J.traces), J.F.u[J.cur], P.nt - 1, s);
        J.finished = true;
        return;
    }
    if (J.phase == 0) {
        // the forward sweep ended in x_{nt-1}: last sample, residual, misfit
        launch_sample(rec_samples(P, J.W.traces),
                      J.W.pool[J.cursor->cur()], P.nt - 1, s);
        launch_residual_misfit(J.W.traces, J.observed, J.W.residual, (long long)P.nrec * P.nt,
                               J.misfit, J.W.partial, s);
        if (J.traces)
            launch_copy(J.traces, J.W.traces, (long long)P.nrec * P.nt, s);
        J.phase = 1;
        J.left = J.cursor->forward_steps() - (P.nt - 1) + P.nt;
        return;
    }
    launch_finalize_dvp(P.dims, J.W.G, nullptr, J.vp, J.dvp, J.W.w[0], J.W.w[1], s);
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
    E->max_slots = max_slots;
    E->max_samples = max_receivers;
    E->ntap = sp->ntap;
    int t = 1;
    while (t * 2 <= max_chunk)
        t *= 2;
    E->tmax = t;
    E->graphs = use_graphs != 0;
    E->slots.resize(max_slots);
    size_t bytes = sizeof(SlotStep) * (size_t)E->tmax * 2 * max_slots;
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
    if (!E || !plan || !slot)
        return fail(STRIDE_E_INVALID_ARG, "NULL engine, plan or slot");
    if (!same_layout(E->dims, plan->dims) || E->R != plan->R || E->ntap != plan->ntap ||
        std::memcmp(&E->cf, &plan->cf, sizeof(StencilCoef)) != 0)
        return fail(STRIDE_E_INVALID_ARG, "plan grid does not match the engine grid");
    if (plan->torder != 2)
        return fail(STRIDE_E_INVALID_ARG, "the engine runs time_order 2 solves only");
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
        for (float* f : {J.W.pool[0], J.W.pool[1], J.W.G, J.W.w[0], J.W.w[1]})
            launch_fill(f, plan->dims.total, 0.f, s);
        J.cursor = std::make_unique<StepCursor>(plan->nt, J.W.snaps, (int)J.W.pool.size());
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

    // per-tick slot tables, active entries packed from row 0, in the pinned
    // staging buffer
    int si = E->stage_i;
    if (E->stage_used[si])
        STRIDE_HIP_TRY(hipEventSynchronize(E->stage_ev[si]));
    SlotStep* H = E->h_stage[si];
    size_t bytes = sizeof(SlotStep) * (size_t)ticks * 2 * E->max_slots;
    std::memset((void*)H, 0, bytes);
    int rows_fwd = 0, rows_adj = 0;
    std::vector<long long> used_ticks(E->max_slots, 0);
    for (int t = 0; t < ticks; ++t) {
        SlotStep* row = H + (size_t)t * 2 * E->max_slots;
        int nf = 0, na = 0;
        for (int j = 0; j < E->max_slots; ++j) {
            SlotJob& J = E->slots[j];
            if (!J.used || J.finished || used_ticks[j] >= J.left)
                continue;
            SlotStep fwd{}, adj{};
            int kind = fill_tick(E, J, &fwd, &adj);
            if (kind < 0)
                return kind;
            if (kind == 1)
                row[nf++] = fwd;
            else
                row[E->max_slots + na++] = adj;
            ++used_ticks[j];
        }
        rows_fwd = std::max(rows_fwd, nf);
        rows_adj = std::max(rows_adj, na);
    }
    // round launch heights up to powers of two so that captured graphs repeat
    auto pow2 = [&](int n) {
        if (n == 0)
            return 0;
        int p = 1;
        while (p < n)
            p *= 2;
        return std::min(p, E->max_slots);
    };
    const int gy_fwd = pow2(rows_fwd), gy_adj = pow2(rows_adj);
    STRIDE_HIP_TRY(hipMemcpyAsync(E->d_table, H, bytes, hipMemcpyHostToDevice, s));
    STRIDE_HIP_TRY(hipEventRecord(E->stage_ev[si], s));
    E->stage_used[si] = true;
    E->stage_i = 1 - si;

    if (E->graphs && s != nullptr) {
        hipGraphExec_t x = nullptr;
        int rc = get_exec(E, ticks, gy_fwd, gy_adj, s, &x);
        if (rc)
            return rc;
        STRIDE_HIP_TRY(hipGraphLaunch(x, s));
    } else {
        launch_chunk(E, ticks, gy_fwd, gy_adj, s);
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
        left += J.cursor->forward_steps() - (J.P->nt - 1) + J.P->nt;
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
