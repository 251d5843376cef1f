// Internal: the plan object, workspace layout, error reporting and the
// step cursor over a checkpointing schedule, shared by the one-shot
// executors (stride_api.cpp) and the batching engine (stride_engine.cpp).
#pragma once

#include <memory>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/stride_hip.h"
#include "common.h"
#include "revolve.h"

struct stride_plan {
    stride_grid_t g;
    int nd, R, nb, nt;
    int torder;          // 2 or 4
    int boundary;        // 0 sponge, 1 perfectly matched layer (forward solves)
    float pml_c0[3];     // PML: second-derivative centre weight / dx_a^2 per axis
    float pml_zmax[3];   // PML: zeta_max per axis
    stride::Dims dims;
    stride::StencilCoef cf;
    stride::Fd1 fd1;     // first-derivative weights in FP64 (medium preparation)
    stride::SpongeCoef sp;
    stride::LaunchShape ls_fwd, ls_adj;
    stride::LaunchShape ls_adjv;         // adjoint steps imaging from a stored v
    double nyquist;      // -(c0 + 2 sum_j cj (-1)^j): largest eigenvalue of -L per axis
    double cellvol;
    int nsrc, nrec;
    int ntap;            // taps per source / receiver (2^nd linear, 8^nd windowed sinc)
    int device;
    void* blob;          // device memory of the tables below
    stride::InjTable src_inj;    // sources, weights / cell volume (blocks of ls_fwd)
    stride::InjTable src_img;    // the same entries, blocks of ls_adj (imaging source term)
    stride::InjTable rec_inj;    // receivers (adjoint injection), weights (blocks of ls_adj)
    stride::InjTable rec_inj_v;  // the same entries, blocks of ls_adjv
    stride::InjTable no_inj;     // no entries (blocks of any shape)
    const long long* rec_idx;
    const float* rec_w;          // receiver sampling
    const long long* src_idx;
    const float* src_w;          // source sampling (adjoint w.r.t. the wavelet), weights / cell volume
};

namespace stride {

// Host-side trace range (rocprofv3 --marker-trace shows it around the work the
// call enqueues); nothing is recorded without a tool attached.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Records the calling thread's last error message and returns `code`.
int fail(int code, const char* fmt, ...);

#define STRIDE_HIP_TRY(expr)                                                                \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::stride::fail(STRIDE_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Layout {
    size_t field;      // bytes per wavefield
    size_t scratch;    // small scalars
    size_t traces;     // nrec * nt floats
    size_t fixed_fwd;  // scratch + k + 2 fields
    size_t fixed_grad; // scratch + k + G + 2 adjoint fields + traces + residual (+ p, q)
    size_t medium;     // scratch + k + 3 wavefields + ndim gamma fields + attenuation
    size_t grad_medium;// medium + G + traces + residual + nt - 1 imaging factors
    size_t grad_medium_fixed; // checkpointed: medium + G + traces + residual + h + scratch u^{m+1}
};

Layout layout_of(const stride_plan& P);

// Views of a gradient workspace:
// [scratch | k | G | w0 | w1 | traces | residual (| p | q, fourth order) | pool...].
struct GradWs {
    unsigned* flags;   // [0] = max vp bits, [1] = bad-value flag
    double* partial;   // misfit partial sums
    float* k;
    float* G;
    float* w[2];
    float* traces;
    float* residual;
    float* p;          // fourth order: k (L u^m + St^m), also the forward steps' p
    float* q;          // fourth order: k L w^{m+1}
    std::vector<float*> pool;   // every field the workspace holds beyond the above
    int peak;                   // fields the binomial schedule uses (pool[0, peak))
    int snaps;
};

int grad_ws(const stride_plan& P, void* ws, size_t bytes, GradWs& W);

// How a gradient runs in a pool of `fields` wavefields (snaps: the binomial
// schedule's snapshot count for that pool).
struct GradPath {
    enum Kind { kFull = 0, kSegmented = 1, kBinomial = 2 };
    int kind = kBinomial;
    std::vector<int> starts;      // segmented: segment starts (0 first; the last segment ends at nt)
    int vbuf = 0;                 // segmented: v fields (the longest segment)
    long long forward_steps = 0;  // forward step launches per gradient
};

GradPath grad_path(const stride_plan& P, long long fields, int snaps);

// Segment starts (0 first) and buffer length of a segmented history for nt
// steps in `fields` pool fields; false when no segmentation fits.
bool make_segments(long long nt, long long fields, std::vector<int>& starts, int& vbuf);

// Segmented history, first sweep: the field that receives u^t from the step
// reading u^{t-1} (fc) and u^{t-2} (fp).  The start states x_{j_k} (k = 1 ..
// K-2) land in their pool pair (pool[vbuf + 2k] = u^{j_k}, pool[vbuf + 2k + 1]
// = u^{j_k - 1}) straight from the steps that produce them, so nothing is
// copied; any other step writes in place of u^{t-2} when that is one of the two
// working fields, else into the working field that does not hold u^{t-1}.
inline float* seg_sweep_out(const GradPath& g, const std::vector<float*>& pool,
                            float* const work[2], const float* fc, const float* fp, int t)
{
    const std::vector<int>& j = g.starts;
    for (int k = 1; k + 1 < (int)j.size(); ++k) {
        if (t == j[k])
            return pool[g.vbuf + 2 * k];
        if (t == j[k] - 1)
            return pool[g.vbuf + 2 * k + 1];
    }
    if (fp == work[0] || fp == work[1])
        return const_cast<float*>(fp);
    return fc == work[0] ? work[1] : work[0];
}

// Views of a forward workspace: [scratch | k | u0 | u1 (| p, fourth order)
// (| psi_a x 2, chi_a per axis, PML)].
struct FwdWs {
    unsigned* flags;
    float* k;
    float* u[2];
    float* p;
    float* psi[2][3];
    float* chi[3];
};

int fwd_ws(const stride_plan& P, void* ws, size_t bytes, FwdWs& F);

// Leapfrog stability bound for a known maximum speed.
int check_cfl(const stride_plan& P, double vmax);

// max(vp) and the bad-value flag read back from the device (one stream sync).
int check_vp(const stride_plan& P, const float* vp, unsigned* flags, hipStream_t s);

StepParams base_params(const stride_plan& P);

// Receiver sampling of a field into out[nrec][nt]; source sampling into out[nsrc][nt].
inline SampleSet rec_samples(const stride_plan& P, float* out)
{
    return SampleSet{P.nrec, P.rec_idx, P.rec_w, out, P.nt, P.ntap, 1.f, 0};
}
inline SampleSet src_samples(const stride_plan& P, float* out)
{
    return SampleSet{P.nsrc, P.src_idx, P.src_w, out, P.nt, P.ntap, 1.f, 0};
}

// One step of a checkpointed gradient solve.
struct StepOp {
    bool reverse;      // adjoint step at `step` (a = u^step, b = u^{step-1}); else forward step
    int step;          // forward: n (u^n -> u^{n+1}); adjoint: m
    int a, b, c;       // pool fields: forward A = u^n, B = u^{n-1}, C = u^{n+1}
    bool first_sweep;  // forward step before the first adjoint step (records traces)
};

// Walks a binomial checkpointing schedule over a reference-counted pool of
// wavefields, one forward or adjoint step at a time.  Store / Free / Restore
// are pure bookkeeping (no copies): a stored state keeps its two fields
// pinned; a step writes in place when its u^{n-1} field is pinned by nothing
// else, and into a free field otherwise (always into a free field with
// in_place false, for steps that read u^{n-1} as a stencil field: the pool
// then needs one field more than the schedule's peak).  Fields 0 and 1 hold
// x_0 = (0, 0).
class StepCursor {
  public:
    StepCursor(int nt, int snaps, int pool_fields, bool in_place = true);
    bool next(StepOp& op);           // false when the schedule is finished
    void unget(const StepOp& op);    // push back one op (to stop before it)
    bool overflow() const { return overflow_; }
    int cur() const { return cur_; }
    long long forward_steps() const { return cs_->stats.forward_steps; }

  private:
    int alloc();
    void release(int f);

    std::shared_ptr<const CachedSchedule> cs_;
    size_t pc_ = 0;
    std::vector<int> ref_;
    std::vector<int> freelist_;
    std::unordered_map<int, std::pair<int, int>> snaps_;
    int cur_ = 0, prev_ = 1, idx_ = 0;
    int target_ = -1;
    bool reversed_ = false;
    bool overflow_ = false;
    bool have_back_ = false;
    bool in_place_ = true;
    StepOp back_{};
};

}  // namespace stride
