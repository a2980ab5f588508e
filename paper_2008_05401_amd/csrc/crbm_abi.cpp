// crbm_abi.cpp -- host side of the C ABI declared in include/crbm.h:
// argument validation, workspace layout, kernel selection and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/crbm.h"
#include "ops.h"
#include "sweep_common.h"
#include "sweep_ising.h"

using namespace crbm;

namespace {

thread_local std::string g_err;

crbm_status fail(crbm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

crbm_status hip_fail(hipError_t e, const char* what)
{
    return fail(CRBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t kLdsLimit = 160 * 1024;
constexpr size_t kJobBytes = 256;
static_assert(sizeof(JobDev) <= kJobBytes, "job descriptor fits its slot");
static_assert(sizeof(crbm_chain_stats) == sizeof(ChainRec), "record layout");

crbm_status check_params(const crbm_params* p)
{
    if (!p) return fail(CRBM_EINVAL, "params is NULL");
    if (p->dense != 0 && p->dense != 1) return fail(CRBM_EINVAL, "dense=%d must be 0 or 1", p->dense);
    const int kmax = p->dense ? 256 : 64;
    if (p->K < 1 || p->K > kmax) return fail(CRBM_EINVAL, "K=%d outside [1,%d]", p->K, kmax);
    if (p->dense && (p->open_cols != 0 || p->n_edge != 0))
        return fail(CRBM_EINVAL, "a dense RBM takes no open_cols or filter banks");
    if (p->C != 1 && p->C != 3) return fail(CRBM_EINVAL, "C=%d must be 1 or 3", p->C);
    if (p->Lw < 1 || p->Lw > 8) return fail(CRBM_EINVAL, "Lw=%d outside [1,8]", p->Lw);
    if (!p->W || !p->hbias || !p->vbias) return fail(CRBM_EINVAL, "W, hbias and vbias must be device pointers");
    if (p->open_cols != 0 && p->open_cols != 1) return fail(CRBM_EINVAL, "open_cols=%d must be 0 or 1", p->open_cols);
    if (p->n_edge < 0 || p->n_edge > 4) return fail(CRBM_EINVAL, "n_edge=%d outside [0,4]", p->n_edge);
    return CRBM_OK;
}

int banks_of(const crbm_params* p) { return 1 + 2 * p->n_edge; }

crbm_status check_lattice(const crbm_params* p, int L)
{
    if (L < 1 || L > 256) return fail(CRBM_EINVAL, "L=%d outside [1,256]", L);
    if (p->Lw > L) return fail(CRBM_EINVAL, "Lw=%d larger than L=%d", p->Lw, L);
    if (2 * p->n_edge > L) return fail(CRBM_EINVAL, "2*n_edge=%d larger than L=%d", 2 * p->n_edge, L);
    if (p->dense && p->Lw != L) return fail(CRBM_EINVAL, "a dense RBM built for L=%d used at L=%d", p->Lw, L);
    return CRBM_OK;
}

enum Kernel { K_GENERIC = 0, K_ISING_FAST = 1 };

struct Plan {
    int kernel;
    int nt;
    int rows;  // rows per lane block (bit-packed kernel)
    size_t lds;
};

// process-wide tile choices for the bit-packed kernel, set by the autotuner
struct TuneEntry {
    int L, K, Lw, rows, nt;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

bool lookup_tuning(int L, int K, int Lw, int* rows, int* nt)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry& t : g_tune)
        if (t.L == L && t.K == K && t.Lw == Lw) {
            *rows = t.rows;
            *nt = t.nt;
            return true;
        }
    return false;
}

crbm_status plan_job(const crbm_params* p, const crbm_batch_desc* d, Plan* out)
{
    crbm_status st = check_params(p);
    if (st != CRBM_OK) return st;
    if (!d) return fail(CRBM_EINVAL, "desc is NULL");
    if (d->target != CRBM_ISING && d->target != CRBM_KITAEV && d->target != CRBM_GIBBS)
        return fail(CRBM_EINVAL, "unknown target %d", d->target);
    st = check_lattice(p, d->L);
    if (st != CRBM_OK) return st;
    if (d->boundary != 0 && d->boundary != 1) return fail(CRBM_EINVAL, "boundary=%d must be 0 or 1", d->boundary);
    if (d->n_chains < 1) return fail(CRBM_EINVAL, "n_chains=%d must be >= 1", d->n_chains);
    if (d->gibbs_k < 1 || d->gibbs_k > 255) return fail(CRBM_EINVAL, "gibbs_k=%d outside [1,255]", d->gibbs_k);
    if (d->burnin_sweeps < 0) return fail(CRBM_EINVAL, "burnin_sweeps must be >= 0");
    if (!(d->mh_band_min >= 0.0)) return fail(CRBM_EINVAL, "mh_band_min must be >= 0");
    if (d->target == CRBM_ISING && p->C != 1) return fail(CRBM_EINVAL, "Ising jobs need C=1 (got %d)", p->C);
    if (d->target == CRBM_KITAEV && d->L > kitaev_max_l())
        return fail(CRBM_EUNSUPPORTED, "Kitaev jobs support L <= %d (got %d)", kitaev_max_l(), d->L);
    if (d->target == CRBM_GIBBS && d->rbm_state)
        return fail(CRBM_EINVAL, "a persistent CRBM replica needs a physical target (got CRBM_GIBBS)");
    Plan pl{};
    const bool plain = p->open_cols == 0 && p->n_edge == 0 && p->dense == 0 && d->boundary == 0;
    if (plain && d->target != CRBM_KITAEV && p->C == 1 && ising_fast_supported(p->K, p->Lw, d->L)) {
        pl.kernel = K_ISING_FAST;
        pl.nt = ising_fast_threads(d->L);
        pl.rows = ising_fast_rows(d->L);
        lookup_tuning(d->L, p->K, p->Lw, &pl.rows, &pl.nt);
        pl.lds = ising_fast_lds_bytes(p->K, p->Lw, d->L);
    } else {
        pl.kernel = K_GENERIC;
        pl.nt = (d->L * d->L * std::max(p->K, p->C) >= 4 * 256) ? 256 : 64;
        // the Kitaev eigen-step is latency-bound: up to N = 64 four waves per chain (one
        // wave tridiagonalises without workgroup barriers, all four bracket the
        // eigenvalues); up to L = 12 eight waves (as fast as sixteen there, with 256
        // VGPRs instead of spilling at 128), sixteen beyond
        if (d->target == CRBM_KITAEV && d->L >= 4) pl.nt = d->L <= 8 ? 256 : (d->L <= 12 ? 512 : 1024);
        pl.lds = generic_lds_bytes(p->K, p->C, p->Lw, d->L, d->target, banks_of(p), p->dense);
    }
    if (pl.lds > kLdsLimit)
        return fail(CRBM_EUNSUPPORTED, "job needs %zu bytes of LDS per chain (limit %zu)", pl.lds, kLdsLimit);
    *out = pl;
    return CRBM_OK;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// workspace: [job descriptor][one record per chain][Kitaev: singular values, n_chains x L^2 doubles]
//            [Kitaev beyond L = 12: eigen-step scratch, n_chains x kitaev_scratch_bytes(L)]
//            [bit-packed Ising kernel: table block of the filters, ising_tab_bytes(K, Lw)]
size_t records_end(int n_chains) { return round_up(kJobBytes + (size_t)n_chains * sizeof(ChainRec), 256); }

size_t eps_end(const crbm_batch_desc* d)
{
    size_t o = records_end(d->n_chains);
    if (d->target == CRBM_KITAEV) o += round_up((size_t)d->n_chains * d->L * d->L * sizeof(double), 256);
    return o;
}

size_t scratch_end(const crbm_batch_desc* d)
{
    size_t o = eps_end(d);
    if (d->target == CRBM_KITAEV) o += round_up((size_t)d->n_chains * kitaev_scratch_bytes(d->L), 256);
    return o;
}

// [... Kitaev regions][bit-packed Ising kernel: the job's table block]
size_t workspace_bytes_for(const crbm_params* p, const crbm_batch_desc* d, const Plan& pl)
{
    size_t o = scratch_end(d);
    if (pl.kernel == K_ISING_FAST) o += round_up(ising_tab_bytes(p->K, p->Lw), 256);
    return o;
}

}  // namespace

struct crbm_ctx {
    crbm_params params;
    crbm_batch_desc desc;
    hipStream_t stream;
    JobDev job;
    JobDev* job_dev;
    ChainRec* rec;
    Plan plan;
    int64_t sweeps;
};

struct crbm_graph {
    hipGraphExec_t exec;
    std::vector<crbm_ctx*> ctxs;
    int64_t sweeps;  // sweeps per chain of one launch of the graph
};

namespace {

crbm_status check_job_list(crbm_ctx* const* ctxs, int n_ctx)
{
    for (int i = 0; i < n_ctx; ++i) {
        if (!ctxs[i]) return fail(CRBM_EINVAL, "job %d is NULL", i);
        if (ctxs[i]->stream != ctxs[0]->stream) return fail(CRBM_EINVAL, "jobs must share one stream");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(CRBM_EINVAL, "job %d listed twice", i);
    }
    return CRBM_OK;
}

crbm_status launch_jobs(crbm_ctx* const* ctxs, int n, int n_sweeps, int mode, hipStream_t s)
{
    // group by kernel variant (and thread count / LDS), larger lattices first, and chunk by
    // MAX_JOBS_PER_LAUNCH
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const Plan& pa = ctxs[a]->plan;
        const Plan& pb = ctxs[b]->plan;
        if (pa.kernel != pb.kernel) return pa.kernel < pb.kernel;
        if (pa.nt != pb.nt) return pa.nt < pb.nt;
        if (pa.rows != pb.rows) return pa.rows < pb.rows;
        if (pa.kernel == K_ISING_FAST && ctxs[a]->params.K != ctxs[b]->params.K) return ctxs[a]->params.K < ctxs[b]->params.K;
        if (pa.kernel == K_ISING_FAST && ctxs[a]->params.Lw != ctxs[b]->params.Lw)
            return ctxs[a]->params.Lw < ctxs[b]->params.Lw;
        // within a launch the larger lattices first: workgroups are dispatched in
        // index order, so the longest ones start earliest (longest-processing-time order)
        return ctxs[a]->desc.L > ctxs[b]->desc.L;
    });
    size_t i = 0;
    while (i < order.size()) {
        const crbm_ctx* c0 = ctxs[order[i]];
        SweepLaunch P;
        memset(&P, 0, sizeof P);
        P.n_sweeps = n_sweeps;
        P.mode = mode;
        size_t lds = 0;
        int blocks = 0;
        int nj = 0;
        while (i < order.size() && nj < MAX_JOBS_PER_LAUNCH) {
            const crbm_ctx* c = ctxs[order[i]];
            if (c->plan.kernel != c0->plan.kernel || c->plan.nt != c0->plan.nt || c->plan.rows != c0->plan.rows) break;
            if (c0->plan.kernel == K_ISING_FAST && (c->params.K != c0->params.K || c->params.Lw != c0->params.Lw)) break;
            P.jobs[nj] = c->job_dev;
            P.block_begin[nj] = blocks;
            blocks += c->desc.n_chains;
            lds = std::max(lds, c->plan.lds);
            ++nj;
            ++i;
        }
        P.block_begin[nj] = blocks;
        P.n_jobs = nj;
        hipError_t e;
        if (c0->plan.kernel == K_ISING_FAST)
            e = launch_ising_fast(P, c0->params.K, c0->params.Lw, c0->plan.rows, blocks, lds, c0->plan.nt, s);
        else
            e = launch_generic(P, blocks, lds, c0->plan.nt, s);
        if (e != hipSuccess) return hip_fail(e, "sweep launch");
    }
    return CRBM_OK;
}

}  // namespace

extern "C" {

size_t crbm_workspace_size(const crbm_params* params, const crbm_batch_desc* desc)
{
    Plan pl;
    if (plan_job(params, desc, &pl) != CRBM_OK) return 0;
    return workspace_bytes_for(params, desc, pl);
}

crbm_status crbm_init(crbm_ctx** out, const crbm_params* params, const crbm_batch_desc* desc, void* stream)
{
    if (!out) return fail(CRBM_EINVAL, "out is NULL");
    *out = nullptr;
    Plan pl;
    crbm_status st = plan_job(params, desc, &pl);
    if (st != CRBM_OK) return st;
    if (!desc->T || !desc->state || !desc->workspace) return fail(CRBM_EINVAL, "T, state and workspace must be device pointers");
    const size_t need = workspace_bytes_for(params, desc, pl);
    if (desc->workspace_bytes < need)
        return fail(CRBM_EBUDGET, "workspace of %zu bytes, %zu needed", desc->workspace_bytes, need);
    if (((uintptr_t)desc->workspace & 255) != 0) return fail(CRBM_EINVAL, "workspace must be 256-byte aligned");
    crbm_ctx* c = new (std::nothrow) crbm_ctx;
    if (!c) return fail(CRBM_EINVAL, "out of host memory");
    c->params = *params;
    c->desc = *desc;
    c->stream = (hipStream_t)stream;
    c->plan = pl;
    c->sweeps = 0;
    c->job_dev = (JobDev*)desc->workspace;
    c->rec = (ChainRec*)((char*)desc->workspace + kJobBytes);
    JobDev& j = c->job;
    memset(&j, 0, sizeof j);
    j.W = params->W;
    j.hb = params->hbias;
    j.vb = params->vbias;
    j.T = desc->T;
    j.state = desc->state;
    j.rbm_state = desc->rbm_state;
    j.rec = c->rec;
    j.eps = desc->target == CRBM_KITAEV ? (double*)((char*)desc->workspace + records_end(desc->n_chains)) : nullptr;
    j.kitA = (desc->target == CRBM_KITAEV && kitaev_scratch_bytes(desc->L) > 0)
                 ? (double*)((char*)desc->workspace + eps_end(desc))
                 : nullptr;
    j.tab = pl.kernel == K_ISING_FAST ? (unsigned char*)desc->workspace + scratch_end(desc) : nullptr;
    j.J0 = desc->J[0];
    j.J1 = desc->J[1];
    j.J2 = desc->J[2];
    j.mh_band_min = desc->mh_band_min;
    j.seed = desc->seed;
    j.K = params->K;
    j.C = params->C;
    j.LW = params->Lw;
    j.target = desc->target;
    j.L = desc->L;
    j.n_chains = desc->n_chains;
    j.gibbs_k = desc->gibbs_k;
    j.burnin = desc->burnin_sweeps;
    j.chain_offset = desc->chain_offset;
    j.init_state = desc->init_state;
    j.open_cols = params->open_cols;
    j.n_edge = params->n_edge;
    j.boundary = desc->boundary;
    j.dense = params->dense;
    hipError_t e = hipMemcpyAsync(c->job_dev, &c->job, sizeof(JobDev), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipMemcpyAsync(job)");
    }
    if (pl.kernel == K_ISING_FAST) {
        // the bit-packed kernel's tables depend on the filters only: built once here
        e = launch_ising_tables(c->job_dev, c->stream);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "table launch");
        }
    }
    SweepLaunch P;
    memset(&P, 0, sizeof P);
    P.jobs[0] = c->job_dev;
    P.block_begin[0] = 0;
    P.block_begin[1] = desc->n_chains;
    P.n_jobs = 1;
    P.mode = MODE_INIT;
    const size_t lds = init_lds(params->K, params->C, params->Lw, desc->L, desc->target, banks_of(params),
                                params->dense);
    if (lds > kLdsLimit) {
        delete c;
        return fail(CRBM_EUNSUPPORTED, "initialisation needs %zu bytes of LDS", lds);
    }
    e = launch_init(P, desc->n_chains, lds, desc->target == CRBM_KITAEV && pl.nt > 256 ? pl.nt : 256, c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "init launch");
    }
    if (pl.kernel == K_ISING_FAST) {
        if (ising_init_fe_lds_bytes(params->K, params->Lw, desc->L) > kLdsLimit) {
            delete c;
            return fail(CRBM_EUNSUPPORTED, "initial free energy needs too much LDS");
        }
        e = launch_ising_init_fe(c->job_dev, desc->n_chains, params->K, params->Lw, desc->L, c->stream);
        if (e != hipSuccess) {
            delete c;
            return hip_fail(e, "free-energy launch");
        }
    }
    *out = c;
    return CRBM_OK;
}

crbm_status crbm_propose_accept(crbm_ctx* ctx, int32_t n_sweeps)
{
    if (!ctx) return fail(CRBM_EINVAL, "ctx is NULL");
    if (n_sweeps < 0) return fail(CRBM_EINVAL, "n_sweeps=%d must be >= 0", n_sweeps);
    if (n_sweeps == 0) return CRBM_OK;
    crbm_ctx* one[1] = {ctx};
    crbm_status st = launch_jobs(one, 1, n_sweeps, MODE_SWEEP, ctx->stream);
    if (st == CRBM_OK) ctx->sweeps += n_sweeps;
    return st;
}

crbm_status crbm_propose_accept_many(crbm_ctx* const* ctxs, int32_t n_ctx, int32_t n_sweeps)
{
    if (!ctxs || n_ctx < 0) return fail(CRBM_EINVAL, "invalid job list");
    if (n_sweeps < 0) return fail(CRBM_EINVAL, "n_sweeps=%d must be >= 0", n_sweeps);
    if (n_ctx == 0 || n_sweeps == 0) return CRBM_OK;
    crbm_status st = check_job_list(ctxs, n_ctx);
    if (st != CRBM_OK) return st;
    st = launch_jobs(ctxs, n_ctx, n_sweeps, MODE_SWEEP, ctxs[0]->stream);
    if (st == CRBM_OK)
        for (int i = 0; i < n_ctx; ++i) ctxs[i]->sweeps += n_sweeps;
    return st;
}

crbm_status crbm_graph_create(crbm_graph** out, crbm_ctx* const* ctxs, int32_t n_ctx, int32_t n_blocks,
                              int32_t sweeps_per_block)
{
    if (!out) return fail(CRBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctxs || n_ctx < 1) return fail(CRBM_EINVAL, "a graph needs at least one job");
    if (n_blocks < 1 || sweeps_per_block < 1)
        return fail(CRBM_EINVAL, "n_blocks=%d and sweeps_per_block=%d must be >= 1", n_blocks, sweeps_per_block);
    crbm_status st = check_job_list(ctxs, n_ctx);
    if (st != CRBM_OK) return st;
    // capture on a private stream: the jobs' stream may be the legacy default
    // stream, which cannot be captured; the kernel nodes do not keep the stream
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e, "hipStreamBeginCapture");
    }
    for (int b = 0; b < n_blocks && st == CRBM_OK; ++b) st = launch_jobs(ctxs, n_ctx, sweeps_per_block, MODE_SWEEP, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (st != CRBM_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    crbm_graph* g = new (std::nothrow) crbm_graph;
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        return fail(CRBM_EINVAL, "out of host memory");
    }
    g->exec = exec;
    g->ctxs.assign(ctxs, ctxs + n_ctx);
    g->sweeps = (int64_t)n_blocks * sweeps_per_block;
    *out = g;
    return CRBM_OK;
}

crbm_status crbm_graph_launch(crbm_graph* g)
{
    if (!g) return fail(CRBM_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, g->ctxs[0]->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    for (crbm_ctx* c : g->ctxs) c->sweeps += g->sweeps;
    return CRBM_OK;
}

crbm_status crbm_graph_destroy(crbm_graph* g)
{
    if (!g) return CRBM_OK;
    hipError_t e = hipGraphExecDestroy(g->exec);
    delete g;
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "hipGraphExecDestroy");
}

crbm_status crbm_tempering_swap(crbm_ctx* ctx, int32_t n_ladders, int32_t round)
{
    if (!ctx) return fail(CRBM_EINVAL, "ctx is NULL");
    if (ctx->desc.target == CRBM_GIBBS) return fail(CRBM_EINVAL, "temperature swaps need a physical target");
    if (n_ladders < 1 || ctx->desc.n_chains % n_ladders != 0)
        return fail(CRBM_EINVAL, "n_ladders=%d must divide n_chains=%d", n_ladders, ctx->desc.n_chains);
    if (round < 0) return fail(CRBM_EINVAL, "round=%d must be >= 0", round);
    const int n_rungs = ctx->desc.n_chains / n_ladders;
    const int q0 = round & 1;
    const int n_rung_pairs = n_rungs - q0 >= 2 ? (n_rungs - q0) / 2 : 0;
    if (n_rung_pairs == 0) return CRBM_OK;
    hipError_t e = launch_tempering_swap(ctx->job_dev, n_rung_pairs * n_ladders, n_ladders, q0, (uint32_t)round,
                                         ctx->desc.target, ctx->stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "tempering swap launch");
}

crbm_status crbm_set_trace(crbm_ctx* ctx, double* trace, int32_t trace_len)
{
    if (!ctx) return fail(CRBM_EINVAL, "ctx is NULL");
    if (trace_len < 0) return fail(CRBM_EINVAL, "trace_len=%d must be >= 0", trace_len);
    ctx->job.trace = (trace && trace_len > 0) ? trace : nullptr;
    ctx->job.trace_len = (trace && trace_len > 0) ? trace_len : 0;
    hipError_t e = hipMemcpyAsync(ctx->job_dev, &ctx->job, sizeof(JobDev), hipMemcpyHostToDevice, ctx->stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "hipMemcpyAsync(job)");
}

crbm_status crbm_autocorr(const double* trace, int32_t n, int32_t len, int32_t start, int32_t max_lag,
                          double c_window, double* out, double* tau, int32_t* window, void* stream)
{
    if (n < 0) return fail(CRBM_EINVAL, "n=%d must be >= 0", n);
    if (len < 1 || len > 8176) return fail(CRBM_EINVAL, "len=%d outside [1,8176]", len);
    if (max_lag < 0 || max_lag >= len) return fail(CRBM_EINVAL, "max_lag=%d outside [0,len)", max_lag);
    if (start < 0) return fail(CRBM_EINVAL, "start=%d must be >= 0", start);
    if (!(c_window > 0.0)) return fail(CRBM_EINVAL, "c_window must be > 0");
    if ((tau == nullptr) != (window == nullptr)) return fail(CRBM_EINVAL, "tau and window are both set or both NULL");
    if (n == 0) return CRBM_OK;
    if (!trace || !out) return fail(CRBM_EINVAL, "trace and out must be device pointers");
    hipError_t e = launch_autocorr(trace, n, len, start % len, max_lag, c_window, out, tau, window,
                                   (hipStream_t)stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "crbm_autocorr launch");
}

crbm_status crbm_read_stats(crbm_ctx* ctx, crbm_chain_stats* out, int32_t on_device)
{
    if (!ctx || !out) return fail(CRBM_EINVAL, "ctx and out must not be NULL");
    const size_t bytes = sizeof(ChainRec) * (size_t)ctx->desc.n_chains;
    hipError_t e;
    if (on_device) {
        e = hipMemcpyAsync(out, ctx->rec, bytes, hipMemcpyDeviceToDevice, ctx->stream);
    } else {
        e = hipMemcpyAsync(out, ctx->rec, bytes, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    if (e != hipSuccess) return hip_fail(e, "crbm_read_stats");
    return CRBM_OK;
}

int64_t crbm_sweeps_done(const crbm_ctx* ctx) { return ctx ? ctx->sweeps : -1; }

crbm_status crbm_destroy(crbm_ctx* ctx)
{
    delete ctx;
    return CRBM_OK;
}

crbm_status crbm_free_energy(const crbm_params* params, const int8_t* x, int32_t B, int32_t L, double* F_out,
                             void* stream)
{
    crbm_status st = check_params(params);
    if (st != CRBM_OK) return st;
    if (B < 0) return fail(CRBM_EINVAL, "B=%d must be >= 0", B);
    st = check_lattice(params, L);
    if (st != CRBM_OK) return st;
    if (B == 0) return CRBM_OK;
    if (!x || !F_out) return fail(CRBM_EINVAL, "x and F_out must be device pointers");
    if (params->dense) {
        hipError_t e = launch_free_energy_dense(params->W, params->hbias, params->vbias, params->K, params->C * L * L,
                                                x, B, F_out, (hipStream_t)stream);
        return e == hipSuccess ? CRBM_OK : hip_fail(e, "crbm_free_energy launch");
    }
    if (free_energy_lds(params->K, params->C, params->Lw, L, banks_of(params)) > kLdsLimit)
        return fail(CRBM_EUNSUPPORTED, "free energy needs too much LDS for L=%d", L);
    hipError_t e = launch_free_energy(params->W, params->hbias, params->vbias, params->K, params->C, params->Lw,
                                      params->open_cols, params->n_edge, x, B, L, F_out, (hipStream_t)stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "crbm_free_energy launch");
}

crbm_status target_energy(int32_t target, const int8_t* x, int32_t B, int32_t C, int32_t L, int32_t boundary,
                          const double J[3], const double* T, int32_t* E_out, double* S_out, void* stream)
{
    if (B < 0) return fail(CRBM_EINVAL, "B=%d must be >= 0", B);
    if (L < 1 || L > 256) return fail(CRBM_EINVAL, "L=%d outside [1,256]", L);
    if (boundary != 0 && boundary != 1) return fail(CRBM_EINVAL, "boundary=%d must be 0 or 1", boundary);
    if (target == CRBM_ISING) {
        if (C != 1) return fail(CRBM_EINVAL, "Ising needs C=1 (got %d)", C);
        if (B == 0) return CRBM_OK;
        if (!x || !E_out) return fail(CRBM_EINVAL, "x and E_out must be device pointers");
        hipError_t e = launch_ising_energy(x, B, L, boundary, E_out, (hipStream_t)stream);
        return e == hipSuccess ? CRBM_OK : hip_fail(e, "target_energy launch");
    }
    if (target == CRBM_KITAEV) {
        if (C != 1 && C != 3) return fail(CRBM_EINVAL, "Kitaev needs C=1 or 3 (got %d)", C);
        if (L > 12) return fail(CRBM_EUNSUPPORTED, "Kitaev supports L <= 12 (got %d)", L);
        if (!J) return fail(CRBM_EINVAL, "J must point to 3 host doubles");
        if (B == 0) return CRBM_OK;
        if (!x || !S_out || !T) return fail(CRBM_EINVAL, "x, T and S_out must be device pointers");
        hipError_t e = launch_kitaev_weight(x, B, C, L, boundary, J[0], J[1], J[2], T, S_out, (hipStream_t)stream);
        return e == hipSuccess ? CRBM_OK : hip_fail(e, "target_energy launch");
    }
    return fail(CRBM_EINVAL, "unknown target %d", target);
}

size_t crbm_grad_workspace_size(const crbm_params* params, int32_t B)
{
    if (check_params(params) != CRBM_OK || B < 0) return 0;
    if (params->dense) {
        const size_t nv = (size_t)params->C * params->Lw * params->Lw;
        return round_up(std::max<size_t>(1, (size_t)B) * (params->K * nv + params->K + nv) * sizeof(double), 256);
    }
    const size_t P = (size_t)banks_of(params) * ((size_t)params->K * params->C * params->Lw * params->Lw + params->K) +
                     params->C;
    return round_up(std::max<size_t>(1, (size_t)B) * P * sizeof(double), 256);
}

crbm_status crbm_grad_static(const crbm_params* params, const int8_t* x, int32_t B, int32_t L, const float* gF,
                             float* dW, float* dhbias, float* dvbias, void* stream)
{
    crbm_status st = check_params(params);
    if (st != CRBM_OK) return st;
    if (B < 0) return fail(CRBM_EINVAL, "B=%d must be >= 0", B);
    const size_t need = crbm_grad_workspace_size(params, B);
    if (need > GRAD_STATIC_BYTES)
        return fail(CRBM_EBUDGET, "crbm_grad_static: %zu bytes of scratch needed, the static scratch holds %zu", need,
                    GRAD_STATIC_BYTES);
    // validate everything crbm_grad would before touching the device
    st = check_lattice(params, L);
    if (st != CRBM_OK) return st;
    void* ptr = nullptr;
    hipError_t e = grad_static_scratch(&ptr);
    if (e != hipSuccess) return hip_fail(e, "crbm_grad_static: scratch address");
    return crbm_grad(params, x, B, L, gF, dW, dhbias, dvbias, ptr, GRAD_STATIC_BYTES, stream);
}

crbm_status crbm_grad(const crbm_params* params, const int8_t* x, int32_t B, int32_t L, const float* gF, float* dW,
                      float* dhbias, float* dvbias, void* workspace, size_t workspace_bytes, void* stream)
{
    crbm_status st = check_params(params);
    if (st != CRBM_OK) return st;
    if (B < 0) return fail(CRBM_EINVAL, "B=%d must be >= 0", B);
    st = check_lattice(params, L);
    if (st != CRBM_OK) return st;
    if (!dW || !dhbias || !dvbias) return fail(CRBM_EINVAL, "gradient outputs must be device pointers");
    if (B > 0 && (!x || !gF)) return fail(CRBM_EINVAL, "x and gF must be device pointers");
    const size_t need = crbm_grad_workspace_size(params, B);
    if (!workspace || workspace_bytes < need)
        return fail(CRBM_EBUDGET, "grad workspace of %zu bytes, %zu needed", workspace_bytes, need);
    if (params->dense) {
        if (grad_dense_lds(params->K, params->C * L * L) > kLdsLimit)
            return fail(CRBM_EUNSUPPORTED, "gradient needs too much LDS for L=%d", L);
        hipError_t e = launch_grad_dense(params->W, params->hbias, params->K, params->C * L * L, x, B, gF,
                                         (double*)workspace, dW, dhbias, dvbias, (hipStream_t)stream);
        return e == hipSuccess ? CRBM_OK : hip_fail(e, "crbm_grad launch");
    }
    if (grad_lds(params->K, params->C, params->Lw, L, banks_of(params)) > kLdsLimit)
        return fail(CRBM_EUNSUPPORTED, "gradient needs too much LDS for L=%d", L);
    hipError_t e = launch_grad(params->W, params->hbias, params->K, params->C, params->Lw, params->open_cols,
                               params->n_edge, x, B, L, gF, (double*)workspace, dW, dhbias, dvbias,
                               (hipStream_t)stream);
    return e == hipSuccess ? CRBM_OK : hip_fail(e, "crbm_grad launch");
}

crbm_status crbm_set_tuning(int32_t L, int32_t K, int32_t Lw, int32_t rows, int32_t threads)
{
    if (!(L == 8 || L == 16 || L == 32 || L == 64 || L == 128 || L == 256))
        return fail(CRBM_EINVAL, "tuning applies to L in {8,...,256} powers of two (got %d)", L);
    if (K < 1 || K > 64 || Lw < 1 || Lw > 6 || Lw > L) return fail(CRBM_EINVAL, "invalid K=%d Lw=%d", K, Lw);
    if (rows != 1 && rows != 2 && rows != 4) return fail(CRBM_EINVAL, "rows=%d must be 1, 2 or 4", rows);
    if (4 * rows > L) return fail(CRBM_EINVAL, "rows=%d too many for L=%d", rows, L);
    if (threads != 64 && threads != 256 && threads != 512 && threads != 1024)
        return fail(CRBM_EINVAL, "threads=%d not in {64,256,512,1024}", threads);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TuneEntry& t : g_tune)
        if (t.L == L && t.K == K && t.Lw == Lw) {
            t.rows = rows;
            t.nt = threads;
            return CRBM_OK;
        }
    g_tune.push_back({L, K, Lw, rows, threads});
    return CRBM_OK;
}

crbm_status crbm_clear_tuning(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
    return CRBM_OK;
}

const char* crbm_last_error(void) { return g_err.c_str(); }

const char* crbm_version(void) { return "crbm-mi355x 0.1 (gfx950)"; }

}  // extern "C"
