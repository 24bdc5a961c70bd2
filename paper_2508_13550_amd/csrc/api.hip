// C ABI entry points: argument checks on the host, then plan/eval/direct.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "common.h"

namespace csfmm {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

static bool valid_kernel(int k) {
    return k >= CSFMM_K_POISSON_LOG && k <= CSFMM_K_SAL;
}

}  // namespace csfmm

using namespace csfmm;

extern "C" {

const char* csfmm_last_error(void) { return g_err; }

int csfmm_plan(const double* targets, int64_t n_t, const double* sources, int64_t n_s,
               int kernel_id, int p, double theta, int leaf_size, unsigned flags, void* stream,
               csfmm_plan_t* out) {
    clear_error();
    if (!out) {
        set_error("out is NULL");
        return CSFMM_E_INVALID;
    }
    *out = nullptr;
    if (!targets || n_t < 1 || n_t > (int64_t(1) << 30)) {
        set_error("targets must be non-NULL with 1 <= n_t <= 2^30 (got %lld)", (long long)n_t);
        return CSFMM_E_INVALID;
    }
    if (sources && (n_s < 1 || n_s > (int64_t(1) << 30))) {
        set_error("1 <= n_s <= 2^30 required (got %lld)", (long long)n_s);
        return CSFMM_E_INVALID;
    }
    if (!valid_kernel(kernel_id)) {
        set_error("unknown kernel id %d", kernel_id);
        return CSFMM_E_INVALID;
    }
    if (p < 1 || p > kMaxDegree) {
        set_error("degree p must be in [1, %d] (got %d)", kMaxDegree, p);
        return CSFMM_E_INVALID;
    }
    if (!(theta > 0.0 && theta < 1.0)) {
        set_error("theta must satisfy 0 < theta < 1 (got %g)", theta);
        return CSFMM_E_INVALID;
    }
    if (leaf_size < 1) {
        set_error("leaf_size must be >= 1 (got %d)", leaf_size);
        return CSFMM_E_INVALID;
    }
    if (flags & ~unsigned(CSFMM_FP32_FORM | CSFMM_SHRINK)) {
        set_error("unknown flags 0x%x", flags);
        return CSFMM_E_INVALID;
    }
    csfmm_plan_s* P = new (std::nothrow) csfmm_plan_s();
    if (!P) {
        set_error("host allocation failed");
        return CSFMM_E_OOM;
    }
    P->nt = n_t;
    P->same = sources == nullptr;
    P->ns = P->same ? n_t : n_s;
    P->kernel = kernel_id;
    P->p = p;
    P->theta = theta;
    P->leaf = leaf_size;
    P->flags = flags;
    P->K = (p + 1) * (p + 1);
    P->KS = int(round_up(P->K, 4));
    int rc = build_plan(P, targets, sources, static_cast<hipStream_t>(stream));
    if (rc != CSFMM_OK) {
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
        delete P;
        return rc;
    }
    *out = P;
    return CSFMM_OK;
}

int csfmm_eval_stages(csfmm_plan_t plan, int kernel_id, const double* weights, double* out,
                      double* wbar, double* psi, double* near, void* stream) {
    clear_error();
    if (!plan || !weights || !out) {
        set_error("plan, weights and out must be non-NULL");
        return CSFMM_E_INVALID;
    }
    if (!valid_kernel(kernel_id)) {
        set_error("unknown kernel id %d", kernel_id);
        return CSFMM_E_INVALID;
    }
    return run_eval(plan, kernel_id, weights, out, wbar, psi, near,
                    static_cast<hipStream_t>(stream));
}

int csfmm_eval_kernel(csfmm_plan_t plan, int kernel_id, const double* weights, double* out,
                      void* stream) {
    return csfmm_eval_stages(plan, kernel_id, weights, out, nullptr, nullptr, nullptr, stream);
}

int csfmm_eval(csfmm_plan_t plan, const double* weights, double* out, void* stream) {
    if (!plan) {
        clear_error();
        set_error("plan is NULL");
        return CSFMM_E_INVALID;
    }
    return csfmm_eval_stages(plan, plan->kernel, weights, out, nullptr, nullptr, nullptr, stream);
}

int csfmm_eval_treecode(csfmm_plan_t plan, int kernel_id, const double* weights, double* out,
                        void* stream) {
    clear_error();
    if (!plan || !weights || !out) {
        set_error("plan, weights and out must be non-NULL");
        return CSFMM_E_INVALID;
    }
    if (!valid_kernel(kernel_id)) {
        set_error("unknown kernel id %d", kernel_id);
        return CSFMM_E_INVALID;
    }
    return run_treecode(plan, kernel_id, weights, out, static_cast<hipStream_t>(stream));
}

namespace {
int direct_entry(const double* targets, int64_t n_t, const double* sources, int64_t n_s,
                 const double* weights, int kernel_id, unsigned flags, double* out, void* stream,
                 bool no_alloc) {
    clear_error();
    if (!targets || !sources || !weights || !out || n_t < 1 || n_s < 1) {
        set_error("direct: non-NULL arrays and n_t, n_s >= 1 required");
        return CSFMM_E_INVALID;
    }
    if (!valid_kernel(kernel_id)) {
        set_error("unknown kernel id %d", kernel_id);
        return CSFMM_E_INVALID;
    }
    if (flags & ~unsigned(CSFMM_FP32_FORM)) {
        set_error("unknown flags 0x%x", flags);
        return CSFMM_E_INVALID;
    }
    return launch_direct(targets, n_t, sources, n_s, weights, kernel_id,
                         (flags & CSFMM_FP32_FORM) != 0, out, static_cast<hipStream_t>(stream),
                         no_alloc);
}
}  // namespace

int csfmm_direct(const double* targets, int64_t n_t, const double* sources, int64_t n_s,
                 const double* weights, int kernel_id, unsigned flags, double* out, void* stream) {
    return direct_entry(targets, n_t, sources, n_s, weights, kernel_id, flags, out, stream, false);
}

int csfmm_direct_noalloc(const double* targets, int64_t n_t, const double* sources, int64_t n_s,
                         const double* weights, int kernel_id, unsigned flags, double* out,
                         void* stream) {
    return direct_entry(targets, n_t, sources, n_s, weights, kernel_id, flags, out, stream, true);
}

int csfmm_plan_destroy(csfmm_plan_t plan) {
    clear_error();
    if (!plan) return CSFMM_OK;
    (void)hipDeviceSynchronize();
    delete plan;
    return CSFMM_OK;
}

int csfmm_plan_stats(csfmm_plan_t plan, csfmm_stats* s) {
    clear_error();
    if (!plan || !s) {
        set_error("plan and stats must be non-NULL");
        return CSFMM_E_INVALID;
    }
    std::memset(s, 0, sizeof(*s));
    s->n_targets = plan->nt;
    s->n_sources = plan->ns;
    s->same_set = plan->same ? 1 : 0;
    s->kernel = plan->kernel;
    s->p = plan->p;
    s->leaf_size = plan->leaf;
    s->theta = plan->theta;
    s->flags = plan->flags;
    s->depth_t = plan->tt.depth;
    s->depth_s = plan->st->depth;
    s->n_cells_t = plan->tt.ncells;
    s->n_cells_s = plan->st->ncells;
    s->n_leaves_t = plan->tt.nleaves;
    s->n_leaves_s = plan->st->nleaves;
    s->max_leaf_t = plan->tt.max_leaf;
    s->pp_sym_pairs = plan->lists.sym.n_own;
    s->pp_one_way = plan->lists.sym.n_one;
    s->pp_close = plan->lists.n_close;
    s->near_wave = csfmm::leaf_wave_path(plan->tt) ? 1 : 0;
    s->n_pp = plan->lists.cnt[kPP];
    s->n_pc = plan->lists.cnt[kPC];
    s->n_cp = plan->lists.cnt[kCP];
    s->n_cc = plan->lists.cnt[kCC];
    s->evals_pp = plan->lists.evals[kPP];
    s->evals_pc = plan->lists.evals[kPC];
    s->evals_cp = plan->lists.evals[kCP];
    s->evals_cc = plan->lists.evals[kCC];
    s->device_bytes = plan->arena.bytes;
    return CSFMM_OK;
}

int64_t csfmm_estimate_bytes(int64_t n_t, int64_t n_s, int p, int leaf_size, unsigned flags) {
    (void)flags;
    if (n_t < 1 || n_s < 0 || p < 1 || p > kMaxDegree || leaf_size < 1) return -1;
    const int64_t K = (p + 1) * (p + 1), KS = round_up(K, 4);
    // cells: at most ~ 4/3 * 4 n / leaf_size per tree (leaves hold > leaf/4 on
    // average for near-uniform points) plus the six roots
    auto cells = [&](int64_t n) { return 6 + (16 * n) / (3 * int64_t(leaf_size)) + 64; };
    const int64_t ct = cells(n_t), cs = n_s ? cells(n_s) : 0;
    int64_t b = 0;
    b += n_t * (5 * 8 + 4) + 6 * 8 * n_t;        // sorted points, local coords, perm, near field
    b += n_s * (5 * 8 + 4 + 8);                  // same for sources, sorted weights
    b += (ct + cs) * (7 * 4 + 4 * 8 + 3 * KS * 8);  // cell arrays, geometry, proxies
    b += cs * KS * 8 + 3 * ct * KS * 8;          // proxy weights, proxy potentials
    b += 4 * (ct + 1) * 4 * 4 + ct * 4 * 160;    // list offsets and entries (~40 per cell per kind)
    b += (ct + cs) * 8 + ct * 2 * 4;             // leaf gaps, PP heads (overlapping, close)
    b += ct * 4 * (3 + 64);                      // symmetric PP split (same-set plans)
    b += 8 * KS * round_up(4 * KS, 16) * 8;      // interpolation operators
    return b;
}

int csfmm_workspace_create(csfmm_plan_t plan, void* stream, csfmm_workspace_t* out) {
    clear_error();
    if (!plan || !out) {
        set_error("plan and out must be non-NULL");
        return CSFMM_E_INVALID;
    }
    return workspace_create(plan, static_cast<hipStream_t>(stream), out);
}

int csfmm_workspace_destroy(csfmm_workspace_t ws) {
    clear_error();
    if (!ws) return CSFMM_OK;
    (void)hipDeviceSynchronize();
    delete ws;
    return CSFMM_OK;
}

int64_t csfmm_workspace_device_bytes(csfmm_workspace_t ws) {
    return ws ? ws->arena.bytes : -1;
}

// The bytes workspace_create allocates for this plan, array by array (each
// starting on a 256-byte boundary of one allocation).
int64_t csfmm_workspace_bytes(csfmm_plan_t plan) {
    if (!plan) return -1;
    auto padded = [](int64_t b) { return (std::max<int64_t>(b, 1) + 255) / 256 * 256; };
    const int64_t d = int64_t(sizeof(double));
    int64_t b = padded(d * plan->ns) + padded(d * plan->st->ncells * plan->KS) +
                padded(d * 3 * plan->tt.ncells * plan->KS) + 2 * padded(d * 3 * plan->nt) +
                padded(int64_t(sizeof(csfmm::ReqView)));
    if (csfmm::sym_path_possible(plan))
        b += padded(csfmm::sym_value_bytes(plan) * plan->lists.sym.n_own * csfmm::kWaveLeaf);
    return b;
}

int csfmm_eval_many(int n_req, const csfmm_plan_t* plans, const csfmm_workspace_t* workspaces,
                    const int* kernel_ids, const double* const* weights, double* const* outs,
                    void* stream) {
    clear_error();
    if (n_req < 0 || (n_req > 0 && (!plans || !workspaces || !weights || !outs))) {
        set_error("eval_many: bad arguments");
        return CSFMM_E_INVALID;
    }
    std::vector<EvalReq> reqs(size_t(n_req > 0 ? n_req : 0));
    for (int r = 0; r < n_req; ++r) {
        csfmm_plan_t P = plans[r];
        csfmm_workspace_t W = workspaces[r];
        const int k = kernel_ids ? kernel_ids[r] : (P ? P->kernel : 0);
        if (!P || !W || W->plan != P || !weights[r] || !outs[r] || !valid_kernel(k)) {
            set_error("eval_many: request %d has a NULL pointer, a workspace of another plan or "
                      "a bad kernel id",
                      r);
            return CSFMM_E_INVALID;
        }
        reqs[r] = EvalReq{P, W, k, weights[r], outs[r]};
    }
    if (n_req == 0) return CSFMM_OK;
    return run_eval_batch(reqs.data(), n_req, static_cast<hipStream_t>(stream));
}

int csfmm_plan_timing(csfmm_plan_t plan, int enable) {
    clear_error();
    if (!plan) {
        set_error("plan is NULL");
        return CSFMM_E_INVALID;
    }
    if (enable < 0 || enable > 2) {
        set_error("timing: enable must be 0, 1 or 2 (got %d)", enable);
        return CSFMM_E_INVALID;
    }
    return timing_enable(plan, enable);
}

int csfmm_plan_timing_read(csfmm_plan_t plan, double* stage_ms, int64_t* n_evals) {
    clear_error();
    if (!plan || !stage_ms || !n_evals) {
        set_error("plan, stage_ms and n_evals must be non-NULL");
        return CSFMM_E_INVALID;
    }
    int rc = timing_collect(plan);
    if (rc != CSFMM_OK) return rc;
    for (int k = 0; k < csfmm_plan_s::Timing::kStages; ++k) stage_ms[k] = plan->timing.sum_ms[k];
    *n_evals = plan->timing.n;
    return CSFMM_OK;
}

int csfmm_plan_cells(csfmm_plan_t plan, int which, int32_t* level, int32_t* face, int32_t* ci,
                     int32_t* cj, int32_t* begin, int32_t* count, int32_t* child0, double* center,
                     double* radius) {
    clear_error();
    if (!plan || (which != 0 && which != 1)) {
        set_error("bad plan or tree selector");
        return CSFMM_E_INVALID;
    }
    const Tree& T = which == 0 ? plan->tt : *plan->st;
    const size_t n = size_t(T.ncells);
    CSFMM_HIP_TRY(hipDeviceSynchronize());
    if (level) CSFMM_HIP_TRY(hipMemcpy(level, T.level, n * 4, hipMemcpyDeviceToHost));
    if (face) CSFMM_HIP_TRY(hipMemcpy(face, T.face, n * 4, hipMemcpyDeviceToHost));
    if (ci) CSFMM_HIP_TRY(hipMemcpy(ci, T.ci, n * 4, hipMemcpyDeviceToHost));
    if (cj) CSFMM_HIP_TRY(hipMemcpy(cj, T.cj, n * 4, hipMemcpyDeviceToHost));
    if (begin) CSFMM_HIP_TRY(hipMemcpy(begin, T.begin, n * 4, hipMemcpyDeviceToHost));
    if (count) CSFMM_HIP_TRY(hipMemcpy(count, T.count, n * 4, hipMemcpyDeviceToHost));
    if (child0) CSFMM_HIP_TRY(hipMemcpy(child0, T.child0, n * 4, hipMemcpyDeviceToHost));
    if (center) CSFMM_HIP_TRY(hipMemcpy(center, T.center, n * 24, hipMemcpyDeviceToHost));
    if (radius) CSFMM_HIP_TRY(hipMemcpy(radius, T.radius, n * 8, hipMemcpyDeviceToHost));
    return CSFMM_OK;
}

int csfmm_plan_proxies(csfmm_plan_t plan, int which, double* proxies) {
    clear_error();
    if (!plan || !proxies || (which != 0 && which != 1)) {
        set_error("bad arguments");
        return CSFMM_E_INVALID;
    }
    const Tree& T = which == 0 ? plan->tt : *plan->st;
    const int K = plan->K, KS = plan->KS;
    std::vector<double> h(size_t(T.ncells) * 3 * KS);
    CSFMM_HIP_TRY(hipDeviceSynchronize());
    CSFMM_HIP_TRY(hipMemcpy(h.data(), T.prox, h.size() * 8, hipMemcpyDeviceToHost));
    for (int64_t c = 0; c < T.ncells; ++c)
        for (int k = 0; k < K; ++k)
            for (int d = 0; d < 3; ++d)
                proxies[(c * K + k) * 3 + d] = h[size_t(c) * 3 * KS + size_t(d) * KS + k];
    return CSFMM_OK;
}

int csfmm_plan_permutation(csfmm_plan_t plan, int which, int64_t* perm) {
    clear_error();
    if (!plan || !perm || (which != 0 && which != 1)) {
        set_error("bad arguments");
        return CSFMM_E_INVALID;
    }
    const Tree& T = which == 0 ? plan->tt : *plan->st;
    std::vector<int32_t> h(size_t(T.n));
    CSFMM_HIP_TRY(hipDeviceSynchronize());
    CSFMM_HIP_TRY(hipMemcpy(h.data(), T.perm, h.size() * 4, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < h.size(); ++k) perm[k] = h[k];
    return CSFMM_OK;
}

int csfmm_plan_list(csfmm_plan_t plan, int kind, int32_t* tgt, int32_t* src, int64_t cap) {
    clear_error();
    if (!plan || kind < 0 || kind > 3 || !tgt || !src) {
        set_error("bad arguments");
        return CSFMM_E_INVALID;
    }
    const int64_t cnt = plan->lists.cnt[kind];
    if (cap < cnt) {
        set_error("list %d has %lld entries, room for %lld", kind, (long long)cnt, (long long)cap);
        return CSFMM_E_INVALID;
    }
    const int nc = plan->tt.ncells;
    std::vector<int32_t> off(size_t(nc) + 1);
    CSFMM_HIP_TRY(hipDeviceSynchronize());
    CSFMM_HIP_TRY(hipMemcpy(off.data(), plan->lists.off[kind], off.size() * 4, hipMemcpyDeviceToHost));
    if (cnt > 0)
        CSFMM_HIP_TRY(hipMemcpy(src, plan->lists.src[kind], size_t(cnt) * 4, hipMemcpyDeviceToHost));
    for (int t = 0; t < nc; ++t)
        for (int e = off[t]; e < off[t + 1]; ++e) tgt[e] = t;
    return CSFMM_OK;
}

}  // extern "C"
