// C-ABI of libddm: setup, factorisation, the DDM step loop of Algorithm 3.1
// (as iterative solver and as FGMRES preconditioner, Sec. 4.2) and the
// single-step entry points.  Host orchestration only; every O(unknowns)
// operation runs in a HIP kernel on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cplx.h"
#include "ddm_internal.h"

using namespace ddm;

namespace ddm {

static hipEvent_t pool_get(ddm_handle *h) {
    if (!h->ev_pool.empty()) {
        hipEvent_t e = h->ev_pool.back();
        h->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

ProfScope::ProfScope(ddm_handle *h_, int cls_, double bytes_, bool on) : h(h_), cls(cls_), bytes(bytes_) {
    if (!on || !h->prof_on) return;
    a = pool_get(h);
    b = pool_get(h);
    if (a && b) (void)hipEventRecord(a, h->stream);
}

ProfScope::~ProfScope() {
    if (!h->prof_on || !a || !b) return;
    (void)hipEventRecord(b, h->stream);
    h->prof_recs.push_back(ddm_handle::ProfRec{a, b, cls, bytes});
}

}  // namespace ddm

namespace {

std::string g_setup_error;

struct HipFail {
    hipError_t e;
    const char *what;
};

#define HIPCHK(expr)                                        \
    do {                                                    \
        hipError_t e_ = (expr);                             \
        if (e_ != hipSuccess) throw HipFail{e_, #expr};     \
    } while (0)

int fail(ddm_handle *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    else g_setup_error = msg;
    return code;
}

int hip_fail(ddm_handle *h, const HipFail &f) {
    char buf[512];
    snprintf(buf, sizeof buf, "HIP error %d (%s) in %s", (int)f.e, hipGetErrorString(f.e), f.what);
    return fail(h, f.e == hipErrorOutOfMemory ? DDM_ENOMEM : DDM_EHIP, buf);
}

// device bytes of one allocation of count elements (zero-sized tables still
// take a 16-byte allocation)
template <typename T> size_t abytes(size_t count) {
    size_t bytes = count * sizeof(T);
    return bytes == 0 ? 16 : bytes;
}

// every device allocation of a handle goes through here, so h->bytes is the
// device memory it holds (and peak_bytes the most it held at once)
template <typename T>
void dalloc(ddm_handle *h, T **p, size_t count) {
    const size_t bytes = abytes<T>(count);
    HIPCHK(hipMalloc((void **)p, bytes));
    h->bytes += bytes;
    h->peak_bytes = std::max(h->peak_bytes, h->bytes);
}

template <typename T>
void dfree(ddm_handle *h, T **p, size_t count) {
    if (!*p) return;
    HIPCHK(hipFree(*p));
    *p = nullptr;
    h->bytes -= abytes<T>(count);
}

size_t elem_size(bool mixed) { return mixed ? sizeof(float2) : sizeof(double2); }

int norm_blocks(const Plan &P) { return stencil_blocks(P); }

constexpr int kDotBlocks = 256;

size_t part_doubles(const Plan &P, int nrhs, int m) {
    size_t a = 2 * (size_t)nrhs * norm_blocks(P);
    size_t b = 2 * (size_t)(m + 1) * nrhs * kDotBlocks;
    size_t c = (size_t)nrhs * 512;
    return std::max(a, std::max(b, c));
}

// Device bytes that ddm_setup allocates for nrhs right-hand sides: the same
// allocations, in the same order and with the same rounding, as ddm_setup
// makes through dalloc (checked there).
size_t setup_bytes(const Plan &P, bool mixed, int nrhs) {
    const size_t es = elem_size(mixed);
    size_t b = 0;
    b += abytes<SubDesc>(P.subs.size()) + abytes<Coef>(P.coef.size()) + abytes<Coef>(P.gcoef.size());
    b += abytes<AxisOwn>(P.aown.size()) + abytes<int2>(P.strip.size() > 0 ? P.strip.size() : 1);
    b += abytes<double>(P.btab.size()) + abytes<SolveItem>(P.items.size()) + abytes<double>((size_t)P.nglob);
    b += abytes<int>((size_t)3 * P.nsub);                           // factorisation status flags
    b += abytes<char>((size_t)P.fel * es);                          // factors
    b += (size_t)(1 + P.ring) * abytes<char>((size_t)nrhs * P.etot * es);  // g + ring
    b += abytes<double2>((size_t)nrhs * P.nglob);                   // residual / operator output
    if (mixed) b += abytes<double2>((size_t)nrhs * P.etot);         // widening scratch
    b += abytes<double>(part_doubles(P, nrhs, 30));
    b += abytes<double>((size_t)4 * nrhs) + abytes<int>((size_t)nrhs);  // norms, active flags
    b += abytes<int>((size_t)4 * P.nsub * sync_tiles_for(nrhs) + 1);  // meeting / read-done / abort flags
    if (chain2_fits(P)) b += abytes<int>((size_t)12 * P.nsub) + abytes<char>(chain2_xbuf_bytes(P));
    b += 2 * abytes<double2>((size_t)nrhs * P.nglob);               // handle-owned f and u (graphs, slots)
    return b;
}

// device bytes of the FGMRES(m) storage for nrhs right-hand sides beyond
// what ddm_setup allocates: the bases V (m + 1 vectors) and Z (m), the dot
// products and coefficients, and the growth of the partial-sum buffer
size_t krylov_bytes(const Plan &P, int nrhs_max, int m) {
    size_t b = abytes<double2>((size_t)(m + 1) * nrhs_max * P.nglob) + abytes<double2>((size_t)m * nrhs_max * P.nglob);
    b += abytes<double2>((size_t)3 * (m + 1) * nrhs_max) + abytes<double2>((size_t)(m + 1) * nrhs_max);
    const size_t need = part_doubles(P, nrhs_max, m), have = part_doubles(P, nrhs_max, 30);
    if (need > have) b += abytes<double>(need) - abytes<double>(have);
    return b;
}

// peak device bytes of a handle: its setup allocations plus the
// factorisation workspace (held during ddm_factor only); plus the FGMRES
// storage for restart m when m > 0
size_t plan_bytes(const Plan &P, bool mixed, int nrhs, int m) {
    size_t b = setup_bytes(P, mixed, nrhs) + factor_ws_bytes(P);
    if (m > 0) b += krylov_bytes(P, nrhs, m);
    return b;
}

void free_all(ddm_handle *h) {
    void *ptrs[] = {h->d_subs, h->d_coef, h->d_gcoef, h->d_aown, h->d_strip, h->d_btab, h->d_k2, h->d_items, h->d_W,
                    h->d_scratch, h->d_flags, h->d_g, h->d_ring[0], h->d_ring[1], h->d_ring[2], h->d_ring[3],
                    h->d_r, h->d_wide, h->d_part, h->d_norm, h->d_active, h->d_V, h->d_Z, h->d_dots,
                    h->d_coef_y, h->d_sync, h->d_sync2, h->d_xbuf, h->d_fin, h->d_uin};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int k = 0; k < 4; ++k)
        if (h->step_graph[k]) (void)hipGraphExecDestroy(h->step_graph[k]);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    for (auto &r : h->prof_recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->h_norm) (void)hipHostFree(h->h_norm);
    if (h->h_dots) (void)hipHostFree(h->h_dots);
}

template <typename T>
const T *ring_at(ddm_handle *h, int s) {  // uhat^s (s >= 1) or null for s <= 0
    return s >= 1 ? (const T *)h->d_ring[s % h->plan.ring] : nullptr;
}

// Run nsteps steps of Algorithm 3.1 with source f (global, complex128) and
// accumulate u += sum_a beta_{0;a} uhat^s_a after every step.  When check is
// given it is called after each step with the per-RHS relative residuals and
// may deactivate RHS (their u is frozen) or request a restart of the
// recursion on a new source (refinement); it returns false to stop.
// One step of Algorithm 3.1 after the first ring generations: transfer,
// local solves, accumulation and (optionally) the residual with its norms
// into d_norm (rcorr: residual-corrected sources, the residual is kept there).
template <typename T>
void enqueue_step(ddm_handle *h, const double2 *f, double2 *u, int nrhs, int s, const double2 *src, bool restrict_src,
                  const double2 *rcorr, bool with_residual) {
    const Plan &P = h->plan;
    T *g = (T *)h->d_g;
    if (restrict_src) HIPCHK((launch_restrict<double2, T>(h, src, g, nrhs)));
    else HIPCHK((launch_transfer<T, T>(h, ring_at<T>(h, s - 1), ring_at<T>(h, s - 2), ring_at<T>(h, s - 3), g, nrhs,
                                       rcorr)));
    T *us = (T *)h->d_ring[s % P.ring];
    HIPCHK(launch_local_solve<T>(h, g, us, nrhs));
    HIPCHK(launch_assemble<T>(h, us, u, nrhs, true, h->d_active));
    if (with_residual)
        HIPCHK(launch_residual(h, f, u, const_cast<double2 *>(rcorr), nrhs, h->d_norm, h->d_norm + nrhs));
}

// Capture the steady-state step of ring phase s % ring as a graph on the
// library's capture stream (every buffer it touches is fixed for that phase).
// Returns false if capture is not possible here (the caller runs eagerly).
template <typename T>
bool step_graph(ddm_handle *h, const double2 *f, double2 *u, int nrhs, int s, const double2 *rcorr) {
    const int phase = s % h->plan.ring;
    if (h->step_graph[phase] && h->step_graph_nrhs[phase] == nrhs) return true;
    if (h->step_graph[phase]) {
        (void)hipGraphExecDestroy(h->step_graph[phase]);
        h->step_graph[phase] = nullptr;
    }
    if (!h->cap_stream && hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking) != hipSuccess) return false;
    hipStream_t keep = h->stream;
    h->stream = h->cap_stream;
    hipGraph_t graph = nullptr;
    bool ok = hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        try {
            enqueue_step<T>(h, f, u, nrhs, s, nullptr, false, rcorr, true);
        } catch (const HipFail &) {
            ok = false;
        }
        hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
        ok = ok && e == hipSuccess && graph;
    }
    h->stream = keep;
    if (ok) ok = hipGraphInstantiate(&h->step_graph[phase], graph, nullptr, nullptr, 0) == hipSuccess;
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    if (!ok) {
        h->step_graph[phase] = nullptr;
        h->use_graphs = false;  // capture unsupported here: stay eager
        return false;
    }
    h->step_graph_nrhs[phase] = nrhs;
    return true;
}

// Run nsteps steps of Algorithm 3.1 with source f (global, complex128) and
// accumulate u += sum_a beta_{0;a} uhat^s_a after every step, followed by the
// residual norms of f - L_h u in d_norm.  check(it, &restart) is then called
// (norms already computed, not yet copied) and may deactivate RHS (their u is
// frozen), request a restart of the recursion on a new source (refinement),
// or return false to stop.  rcorr: residual-corrected sources (the residual
// is written there every step).  graphs: steady-state steps replay a
// captured hipGraph (f and u must then be buffers that stay fixed).
template <typename T, typename Check>
void run_steps(ddm_handle *h, const double2 *f, double2 *u, int nrhs, int nsteps, Check check,
               const double2 *rcorr = nullptr, bool graphs = false) {
    const Plan &P = h->plan;
    const double2 *src = f;
    int s = 0;
    for (int it = 1; it <= nsteps; ++it) {
        ++s;
        bool done = false;
        if (graphs && h->use_graphs && !h->prof_on && s > P.ring && step_graph<T>(h, f, u, nrhs, s, rcorr)) {
            HIPCHK(hipGraphLaunch(h->step_graph[s % P.ring], h->stream));
            ++h->graph_launches;
            done = true;
        }
        if (!done) enqueue_step<T>(h, f, u, nrhs, s, src, s == 1, rcorr, true);
        const double2 *restart_src = nullptr;
        if (!check(it, &restart_src)) break;
        if (restart_src) {
            src = restart_src;
            s = 0;
        }
    }
}

// step loop without residuals (the FGMRES preconditioner M_K)
template <typename T>
void run_steps_plain(ddm_handle *h, const double2 *f, double2 *u, int nrhs, int nsteps) {
    for (int s = 1; s <= nsteps; ++s) enqueue_step<T>(h, f, u, nrhs, s, f, s == 1, nullptr, false);
}

void set_active(ddm_handle *h, const std::vector<int> &act) {
    HIPCHK(hipMemcpyAsync(h->d_active, act.data(), act.size() * sizeof(int), hipMemcpyHostToDevice, h->stream));
}

// fetch the norms a step left in d_norm: relres per RHS
void fetch_norms(ddm_handle *h, int nrhs, std::vector<double> &rel, std::vector<double> *fn = nullptr) {
    HIPCHK(hipMemcpyAsync(h->h_norm, h->d_norm, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    rel.resize(nrhs);
    if (fn) fn->resize(nrhs);
    for (int q = 0; q < nrhs; ++q) {
        double rn = std::sqrt(h->h_norm[q]), fnq = std::sqrt(h->h_norm[nrhs + q]);
        rel[q] = fnq > 0 ? rn / fnq : rn;
        if (fn) (*fn)[q] = fnq;
    }
}

// relres per RHS of u for source f; fills h->h_norm[0..2 nrhs)
void residual_host(ddm_handle *h, const double2 *f, const double2 *u, double2 *r, int nrhs, std::vector<double> &rel,
                   std::vector<double> *fn = nullptr) {
    HIPCHK(launch_residual(h, f, u, r, nrhs, h->d_norm, h->d_norm + nrhs));
    HIPCHK(hipMemcpyAsync(h->h_norm, h->d_norm, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    rel.resize(nrhs);
    if (fn) fn->resize(nrhs);
    for (int q = 0; q < nrhs; ++q) {
        double rn = std::sqrt(h->h_norm[q]), fnq = std::sqrt(h->h_norm[nrhs + q]);
        rel[q] = fnq > 0 ? rn / fnq : rn;
        if (fn) (*fn)[q] = fnq;
    }
}

// The chain substitution raises a sticky flag when the wait for the partner
// chain exceeded its spin bound; read and clear it (synchronises the stream).
int check_abort(ddm_handle *h) {
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, abort_flag_ptr(h), sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (flag) {
        HIPCHK(hipMemsetAsync(abort_flag_ptr(h), 0, sizeof(int), h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        return fail(h, DDM_EHIP, "substitution: the wait for the partner chain exceeded its spin bound; results invalid");
    }
    return DDM_OK;
}

bool slots_busy(const ddm_handle *h) {
    for (int s : h->slot_steps)
        if (s >= 0) return true;
    return false;
}

int check_args(ddm_handle *h, int nrhs) {
    if (!h) return DDM_EINVAL;
    if (nrhs < 1 || nrhs > h->nrhs_max) {
        char buf[128];
        snprintf(buf, sizeof buf, "nrhs=%d outside [1, %d]", nrhs, h->nrhs_max);
        return fail(h, DDM_EINVAL, buf);
    }
    return DDM_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------------------
// Stationary DDM (Sec. 4.2.1), FP64 or mixed with residual restarts
// ---------------------------------------------------------------------------
template <typename T>
int solve_stationary(ddm_handle *h, const double2 *f, double2 *u, int nrhs, const ddm_solve_opts &o,
                     ddm_rhs_info *info) {
    const Plan &P = h->plan;
    double t0 = now_s();
    // graph path: iterate on handle-owned copies of f and u so that captured
    // steps stay valid across calls
    const bool graphs = h->use_graphs && !h->prof_on;
    const double2 *fout = f;
    double2 *uout = u;
    const size_t vbytes = (size_t)nrhs * P.nglob * sizeof(double2);
    if (graphs) {
        HIPCHK(hipMemcpyAsync(h->d_fin, f, vbytes, hipMemcpyDeviceToDevice, h->stream));
        f = h->d_fin;
        u = h->d_uin;
    }
    HIPCHK(launch_fill_zero(u, (long long)vbytes, h->stream));
    std::vector<int> act(nrhs, 1);
    set_active(h, act);
    std::vector<double> rel, fn, best(nrhs, 1e300), last_gain_rel(nrhs, 1.0);
    std::vector<int> steps(nrhs, 0), status(nrhs, DDM_ENOCONV), since_gain(nrhs, 0);
    std::vector<double> secs(nrhs, 0.0), final_rel(nrhs, 1.0);
    // restart on the residual after refine_every steps without a 2x gain
    // (opt-in: the residual-corrected sources of the mixed path do not stall)
    const int refine_every = o.refine_every;
    double2 *rsrc = h->d_r;  // residual (corrected sources) / restart source
    const int check_every = std::max(1, o.check_every);
    auto check = [&](int it, const double2 **restart) -> bool {
        // between checks the steps are only enqueued (no host synchronisation)
        if (it % check_every != 0 && it < o.maxiter) return true;
        fetch_norms(h, nrhs, rel, &fn);
        bool all = true, changed = false;
        bool stalled = false;
        for (int q = 0; q < nrhs; ++q) {
            if (!act[q]) continue;
            steps[q] = it;
            final_rel[q] = rel[q];
            if (!std::isfinite(rel[q])) { status[q] = DDM_EDIVERGED; act[q] = 0; changed = true; continue; }
            if (rel[q] <= o.tol) {
                status[q] = DDM_OK; act[q] = 0; changed = true;
                secs[q] = now_s() - t0;
                continue;
            }
            if (rel[q] > 1e6 * best[q]) { status[q] = DDM_EDIVERGED; act[q] = 0; changed = true; continue; }
            if (rel[q] < best[q]) best[q] = rel[q];
            if (rel[q] < 0.5 * last_gain_rel[q]) { last_gain_rel[q] = rel[q]; since_gain[q] = 0; }
            else if (refine_every > 0 && ++since_gain[q] >= refine_every) stalled = true;
            all = false;
        }
        if (changed) set_active(h, act);
        if (all || it >= o.maxiter) return false;
        if (h->mixed && stalled) {
            // iterative refinement: restart the complex64 recursion on the FP64
            // residual r = f - L u (already in rsrc); u keeps accumulating
            for (int q = 0; q < nrhs; ++q) { since_gain[q] = 0; last_gain_rel[q] = rel[q]; }
            *restart = rsrc;
        }
        return true;
    };
    run_steps<T>(h, f, u, nrhs, o.maxiter, check, h->mixed ? rsrc : nullptr, graphs);
    if (graphs) HIPCHK(hipMemcpyAsync(uout, u, vbytes, hipMemcpyDeviceToDevice, h->stream));
    (void)fout;
    HIPCHK(hipStreamSynchronize(h->stream));
    int worst = DDM_OK;
    double t1 = now_s();
    for (int q = 0; q < nrhs; ++q) {
        if (status[q] != DDM_OK) secs[q] = t1 - t0;
        if (info) {
            info[q].iters = steps[q];
            info[q].local_solves = steps[q];
            info[q].relres = final_rel[q];
            info[q].seconds = secs[q];
            info[q].status = status[q];
        }
        if (status[q] > worst) worst = status[q];
    }
    return worst;
}

// ---------------------------------------------------------------------------
// FGMRES(m) right-preconditioned by K DDM steps (Sec. 4.2.2), lockstep over
// the RHS of a batch, classical Gram-Schmidt applied twice, FP64.
// ---------------------------------------------------------------------------
void ensure_krylov(ddm_handle *h, int m, int nrhs) {
    if (h->d_V && h->krylov_m >= m && h->krylov_nrhs >= nrhs) return;
    const Plan &P = h->plan;
    const int km = h->krylov_m, kn = h->krylov_nrhs;
    dfree(h, &h->d_V, (size_t)(km + 1) * kn * P.nglob);
    dfree(h, &h->d_Z, (size_t)km * kn * P.nglob);
    dfree(h, &h->d_dots, (size_t)3 * (km + 1) * kn);
    dfree(h, &h->d_coef_y, (size_t)(km + 1) * kn);
    if (h->h_dots) { HIPCHK(hipHostFree(h->h_dots)); h->h_dots = nullptr; }
    h->krylov_m = h->krylov_nrhs = 0;
    long long n = P.nglob;
    size_t need = part_doubles(P, std::max(nrhs, h->nrhs_max), m);
    // the basis lives beside the factors: respect the handle's HBM budget
    size_t grow = abytes<double2>((size_t)(m + 1) * nrhs * n) + abytes<double2>((size_t)m * nrhs * n) +
                  abytes<double2>((size_t)3 * (m + 1) * nrhs) + abytes<double2>((size_t)(m + 1) * nrhs) +
                  (need > h->part_cap ? abytes<double>(need) - abytes<double>(h->part_cap) : 0);
    if (h->prob.hbm_budget_bytes > 0 && h->bytes + grow > h->prob.hbm_budget_bytes)
        throw HipFail{hipErrorOutOfMemory, "FGMRES basis beyond the HBM budget"};
    if (need > h->part_cap) {
        dfree(h, &h->d_part, h->part_cap);
        dalloc(h, &h->d_part, need);
        h->part_cap = need;
    }
    dalloc(h, &h->d_V, (size_t)(m + 1) * nrhs * n);
    dalloc(h, &h->d_Z, (size_t)m * nrhs * n);
    dalloc(h, &h->d_dots, (size_t)3 * (m + 1) * nrhs);
    dalloc(h, &h->d_coef_y, (size_t)(m + 1) * nrhs);
    // the update x += Z y reads only the basis vectors a cycle formed, but
    // start from zeros so no stale bits can ever reach it
    HIPCHK(launch_fill_zero(h->d_Z, (long long)m * nrhs * n * sizeof(double2), h->stream));
    HIPCHK(hipHostMalloc((void **)&h->h_dots, (size_t)3 * (m + 1) * nrhs * sizeof(double2), hipHostMallocDefault));
    h->krylov_m = m;
    h->krylov_nrhs = nrhs;
}

template <typename T>
int solve_fgmres(ddm_handle *h, const double2 *f, double2 *x, int nrhs, const ddm_solve_opts &o, ddm_rhs_info *info) {
    using cd = std::complex<double>;
    const Plan &P = h->plan;
    const long long n = P.nglob;
    const int m = o.restart > 0 ? o.restart : 30;
    int K = o.K > 0 ? o.K : (P.N[0] + P.N[1] + P.N[2] - (3 - P.dim));
    double t0 = now_s();
    ensure_krylov(h, m, nrhs);
    // V_j of RHS q at d_V + (j * nrhs + q) * n; vstride = nrhs * n, ld = n
    const long long vstride = (long long)nrhs * n;
    double2 *V = h->d_V, *Z = h->d_Z, *w = h->d_r;
    HIPCHK(launch_fill_zero(x, (long long)nrhs * n * sizeof(double2), h->stream));
    std::vector<int> done(nrhs, 0), its(nrhs, 0), status(nrhs, DDM_ENOCONV);
    std::vector<double> fnorm(nrhs, 0.0), rel(nrhs, 1.0);
    std::vector<cd> H((size_t)nrhs * (m + 1) * m), cs((size_t)nrhs * m), sn((size_t)nrhs * m), gv((size_t)nrhs * (m + 1));
    std::vector<int> jr(nrhs), fin(nrhs);
    std::vector<double2> yh((size_t)nrhs * m);
    std::vector<int> ones(nrhs, 1);
    int total = 0;
    bool first = true;
    while (true) {
        // r0 = f - A x  ->  V_0, norms
        std::vector<double> rr, ff;
        residual_host(h, f, x, V, nrhs, rr, &ff);
        if (first) {
            for (int q = 0; q < nrhs; ++q) {
                fnorm[q] = ff[q];
                if (!std::isfinite(ff[q])) throw std::string("non-finite source");
                if (fnorm[q] == 0) { done[q] = 1; status[q] = DDM_OK; rel[q] = 0; }
            }
            first = false;
        }
        bool all = true;
        for (int q = 0; q < nrhs; ++q) {
            if (done[q]) continue;
            rel[q] = rr[q];
            if (rr[q] <= o.tol) { done[q] = 1; status[q] = DDM_OK; continue; }
            if (its[q] >= o.maxiter) continue;
            all = false;
        }
        if (all || total >= o.maxiter) break;
        // V_0 /= ||r0|| (scale factors = squared residual norms in d_norm)
        HIPCHK(launch_scale(V, V, h->d_norm, n, nrhs, n, h->stream));
        for (int q = 0; q < nrhs; ++q) {
            jr[q] = 0;
            fin[q] = done[q] || its[q] >= o.maxiter;
            std::fill(gv.begin() + (size_t)q * (m + 1), gv.begin() + (size_t)(q + 1) * (m + 1), cd(0));
            gv[(size_t)q * (m + 1)] = cd(std::sqrt(h->h_norm[q]), 0.0);
        }
        for (int j = 0; j < m; ++j) {
            double2 *vj = V + j * vstride, *zj = Z + j * vstride;
            // z_j = M_K(v_j): K DDM steps from a zero state, output sum beta0 U
            set_active(h, ones);
            HIPCHK(launch_fill_zero(zj, vstride * (long long)sizeof(double2), h->stream));
            run_steps_plain<T>(h, vj, zj, nrhs, K);
            HIPCHK(launch_apply(h, zj, w, nrhs));
            double2 *h1 = h->d_dots, *h2 = h->d_dots + (size_t)(m + 1) * nrhs;
            double *hn = (double *)(h->d_dots + (size_t)2 * (m + 1) * nrhs);
            // dots are laid out [rhs][i] for i <= j
            HIPCHK(launch_dots(V, j + 1, vstride, w, n, nrhs, n, h1, h->d_part, kDotBlocks, h->stream));
            HIPCHK(launch_axpy_multi(w, V, j + 1, vstride, h1, -1.0, n, nrhs, n, h->stream));
            HIPCHK(launch_dots(V, j + 1, vstride, w, n, nrhs, n, h2, h->d_part, kDotBlocks, h->stream));
            HIPCHK(launch_axpy_multi(w, V, j + 1, vstride, h2, -1.0, n, nrhs, n, h->stream));
            HIPCHK(launch_norm2(h, w, n, nrhs, n, hn));
            HIPCHK(launch_scale(V + (j + 1) * vstride, w, hn, n, nrhs, n, h->stream));
            HIPCHK(hipMemcpyAsync(h->h_dots, h->d_dots, (size_t)3 * (m + 1) * nrhs * sizeof(double2),
                                  hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            ++total;
            const double2 *H1 = h->h_dots, *H2 = h->h_dots + (size_t)(m + 1) * nrhs;
            const double *HN = (const double *)(h->h_dots + (size_t)2 * (m + 1) * nrhs);
            bool cycle_done = true;
            for (int q = 0; q < nrhs; ++q) {
                if (fin[q]) continue;
                cd *Hq = &H[(size_t)q * (m + 1) * m];
                for (int i = 0; i <= j; ++i)
                    Hq[i * m + j] = cd(H1[q * (j + 1) + i].x + H2[q * (j + 1) + i].x,
                                       H1[q * (j + 1) + i].y + H2[q * (j + 1) + i].y);
                double hnq = std::sqrt(HN[q]);
                Hq[(j + 1) * m + j] = cd(hnq, 0);
                cd *c = &cs[(size_t)q * m], *sN = &sn[(size_t)q * m], *g = &gv[(size_t)q * (m + 1)];
                for (int i = 0; i < j; ++i) {
                    cd a = Hq[i * m + j], b = Hq[(i + 1) * m + j];
                    Hq[i * m + j] = std::conj(c[i]) * a + std::conj(sN[i]) * b;
                    Hq[(i + 1) * m + j] = -sN[i] * a + c[i] * b;
                }
                cd a = Hq[j * m + j], b = Hq[(j + 1) * m + j];
                double rn = std::sqrt(std::norm(a) + std::norm(b));
                if (rn == 0) { c[j] = 1; sN[j] = 0; }
                else { c[j] = a / rn; sN[j] = b / rn; }
                Hq[j * m + j] = rn;
                Hq[(j + 1) * m + j] = 0;
                g[j + 1] = -sN[j] * g[j];
                g[j] = std::conj(c[j]) * g[j];
                jr[q] = j + 1;
                its[q] += 1;
                double est = std::abs(g[j + 1]) / fnorm[q];
                if (est <= o.tol || hnq == 0 || its[q] >= o.maxiter) fin[q] = 1;
                else cycle_done = false;
            }
            if (cycle_done) break;
        }
        // x_q += Z y_q, y from the triangular system of the cycle; only the
        // nvec basis vectors this cycle formed enter the update
        int nvec = 0;
        for (int q = 0; q < nrhs; ++q) nvec = std::max(nvec, done[q] ? 0 : jr[q]);
        for (int q = 0; q < nrhs; ++q) {
            std::vector<cd> y(m, cd(0));
            int jq = done[q] ? 0 : jr[q];
            cd *Hq = &H[(size_t)q * (m + 1) * m];
            cd *g = &gv[(size_t)q * (m + 1)];
            for (int i = jq - 1; i >= 0; --i) {
                cd s = g[i];
                for (int k = i + 1; k < jq; ++k) s -= Hq[i * m + k] * y[k];
                y[i] = s / Hq[i * m + i];
            }
            for (int i = 0; i < nvec; ++i) yh[(size_t)q * nvec + i] = make_double2(y[i].real(), y[i].imag());
        }
        if (nvec > 0) {
            HIPCHK(hipMemcpyAsync(h->d_coef_y, yh.data(), (size_t)nrhs * nvec * sizeof(double2), hipMemcpyHostToDevice,
                                  h->stream));
            HIPCHK(launch_axpy_multi(x, Z, nvec, vstride, h->d_coef_y, 1.0, n, nrhs, n, h->stream));
        }
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    double t1 = now_s();
    int worst = DDM_OK;
    for (int q = 0; q < nrhs; ++q) {
        if (info) {
            info[q].iters = its[q];
            info[q].local_solves = its[q] * K;
            info[q].relres = rel[q];
            info[q].seconds = t1 - t0;
            info[q].status = status[q];
        }
        if (status[q] > worst) worst = status[q];
    }
    return worst;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

int ddm_profile_enable(ddm_handle *h, int on) {
    if (!h) return DDM_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    for (auto &r : h->prof_recs) { h->ev_pool.push_back(r.a); h->ev_pool.push_back(r.b); }
    h->prof_recs.clear();
    h->prof_on = on != 0;
    return DDM_OK;
}

int ddm_profile_read(ddm_handle *h, ddm_profile *out) {
    if (!h || !out) return DDM_EINVAL;
    memset(out, 0, sizeof(*out));
    if (hipStreamSynchronize(h->stream) != hipSuccess) return fail(h, DDM_EHIP, "stream synchronize failed");
    for (auto &r : h->prof_recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess && r.cls >= 0 && r.cls < DDM_K_NCLASS) {
            out->launches[r.cls] += 1;
            out->ms[r.cls] += ms;
            out->bytes[r.cls] += r.bytes;
        }
    }
    return DDM_OK;
}

// Default substitution variant: the split chains when at most 4 RHS share a
// launch (one pass over the inverses either way), the blocks are large enough
// for half a block's stream to outweigh the per-block exchange (>= 128
// unknowns; on 68-unknown blocks the split launch measured 40% slower) and
// the plan admits them; else one workgroup per chain (its 8 / 16-RHS tiles
// stream every inverse once for up to 16 RHS); else the per-line launches.
static int default_variant(const ddm_handle *h) {
    if (h->nrhs_max >= kMmaMinRhs && solve_variant_ok(h->plan, kSolveMma)) return kSolveMma;
    if (h->nrhs_max <= 4 && h->plan.bs_max >= 128 && h->d_xbuf && solve_variant_ok(h->plan, kSolveChain2))
        return kSolveChain2;
    return solve_variant_ok(h->plan, kSolveChain) ? kSolveChain : kSolvePerLine;
}

// captured step graphs hold kernel choices and arguments: drop them when a
// setting they bake in changes
static void drop_step_graphs(ddm_handle *h) {
    for (int k = 0; k < 4; ++k)
        if (h->step_graph[k]) { (void)hipGraphExecDestroy(h->step_graph[k]); h->step_graph[k] = nullptr; }
}

// Select a substitution variant.  The matrix-core variant reads the inverses
// in its own operand order: switching to or from it re-runs the
// factorisation in the other order (when the handle was factored).
static int select_variant(ddm_handle *h, int variant) {
    if (variant != h->solve_variant) drop_step_graphs(h);
    h->solve_variant = variant;
    const bool mma = variant == kSolveMma;
    if (mma == h->plan.mma) return DDM_OK;
    h->plan.mma = mma;
    if (!h->factored) return DDM_OK;
    h->factored = false;
    return ddm_factor(h);
}

int ddm_set_solve_variant(ddm_handle *h, int variant) {
    if (!h) return DDM_EINVAL;
    if (variant < 0 || variant >= kSolveNVariants || !solve_variant_ok(h->plan, variant))
        return fail(h, DDM_EINVAL, "substitution variant does not apply to this problem");
    return select_variant(h, variant);
}

int ddm_set_transfer_form(ddm_handle *h, int form) {
    if (!h) return DDM_EINVAL;
    if (form != DDM_TRANSFER_DIRECT && form != DDM_TRANSFER_PHI) return fail(h, DDM_EINVAL, "unknown transfer form");
    if (form == DDM_TRANSFER_PHI) {
        int split = 0;
        for (int d = 0; d < h->plan.dim; ++d) split += h->plan.N[d] > 1;
        if (split > 1)
            return fail(h, DDM_EINVAL,
                        "the Phi form of the transferred source needs subdomains along one axis only: with corner "
                        "transfers the local sources do not vanish where the cut-offs vary");
    }
    if (form != h->transfer_form) drop_step_graphs(h);
    h->transfer_form = form;
    return DDM_OK;
}

int ddm_set_factor_layout(ddm_handle *h, int twisted) {
    if (!h) return DDM_EINVAL;
    if (twisted && !solve_variant_ok(h->plan, kSolveChain))
        return fail(h, DDM_EINVAL, "the twisted layout needs the chain substitution (block size <= 256)");
    if (twisted && 2 * h->plan.nsub > h->plan.ncu)
        return fail(h, DDM_EINVAL, "the twisted layout needs one resident workgroup per chain (2 nsub <= compute units)");
    (void)hipStreamSynchronize(h->stream);
    plan_set_twist(&h->plan, twisted != 0);
    if (hipMemcpy(h->d_subs, h->plan.subs.data(), h->plan.subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice) !=
        hipSuccess)
        return fail(h, DDM_EHIP, "descriptor upload failed");
    h->factored = false;
    for (int k = 0; k < 4; ++k)
        if (h->step_graph[k]) { (void)hipGraphExecDestroy(h->step_graph[k]); h->step_graph[k] = nullptr; }
    if (!solve_variant_ok(h->plan, h->solve_variant)) h->solve_variant = default_variant(h);
    h->plan.mma = h->solve_variant == kSolveMma;
    return DDM_OK;
}

int ddm_set_graphs(ddm_handle *h, int on) {
    if (!h) return DDM_EINVAL;
    h->use_graphs = on != 0;
    return DDM_OK;
}

long ddm_graph_launches(const ddm_handle *h) { return h ? h->graph_launches : -1; }

int ddm_get_solve_variant(const ddm_handle *h) { return h ? h->solve_variant : -1; }

int ddm_set_spin_limit(ddm_handle *h, int limit) {
    if (!h || limit < 1) return DDM_EINVAL;
    if (limit != h->spin_limit) drop_step_graphs(h);
    h->spin_limit = limit;
    return DDM_OK;
}

int ddm_set_chain_tile(ddm_handle *h, int rt) {
    if (!h) return DDM_EINVAL;
    if (rt != 0 && rt != 4 && rt != 8 && rt != 16) return fail(h, DDM_EINVAL, "chain RHS tile must be 0, 4, 8 or 16");
    if (rt != h->chain_tile) drop_step_graphs(h);
    h->chain_tile = rt;
    return DDM_OK;
}

int ddm_time_local_solve(ddm_handle *h, int nrhs, int reps, double *ms) {
    int st = check_args(h, nrhs);
    if (st) return st;
    if (!ms || reps < 1) return fail(h, DDM_EINVAL, "ms must be non-null and reps >= 1");
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_time_local_solve before ddm_factor");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const size_t es = elem_size(h->mixed);
        HIPCHK(launch_fill_zero(h->d_g, (long long)nrhs * h->plan.etot * es, h->stream));
        h->g_clean_rows = 0;
        auto once = [&]() {
            HIPCHK(h->mixed ? launch_local_solve<float2>(h, (const float2 *)h->d_g, (float2 *)h->d_ring[0], nrhs)
                            : launch_local_solve<double2>(h, (const double2 *)h->d_g, (double2 *)h->d_ring[0], nrhs));
        };
        once();  // warm-up
        HIPCHK(hipEventRecord(e0, h->stream));
        for (int r = 0; r < reps; ++r) once();
        HIPCHK(hipEventRecord(e1, h->stream));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        *ms = t / reps;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } catch (const HipFail &e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return hip_fail(h, e);
    }
    return check_abort(h);
}

int ddm_autotune(ddm_handle *h, int nrhs, int reps, double *times_ms) {
    int st = check_args(h, nrhs);
    if (st) return st;
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_autotune before ddm_factor");
    if (reps < 1) reps = 1;
    const Plan &P = h->plan;
    int best = -1, keep = h->solve_variant;
    double best_ms = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    try {
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        size_t es = elem_size(h->mixed);
        HIPCHK(launch_fill_zero(h->d_g, (long long)nrhs * P.etot * es, h->stream));
        h->g_clean_rows = 0;
        // the variants that read the current layout of the inverses first,
        // then the others (one re-factorisation between the two groups)
        std::vector<int> order;
        for (int pass = 0; pass < 2; ++pass)
            for (int v = 0; v < kSolveNVariants; ++v)
                if (((v == kSolveMma) == h->plan.mma) == (pass == 0)) order.push_back(v);
        for (int v : order) {
            if (times_ms) times_ms[v] = -1.0;
            if (!solve_variant_ok(P, v)) continue;
            int sv = select_variant(h, v);
            if (sv != DDM_OK) {
                (void)select_variant(h, keep);
                return sv;
            }
            hipError_t e = h->mixed ? launch_local_solve<float2>(h, (const float2 *)h->d_g, (float2 *)h->d_ring[0], nrhs)
                                    : launch_local_solve<double2>(h, (const double2 *)h->d_g, (double2 *)h->d_ring[0], nrhs);
            if (e != hipSuccess) { (void)hipGetLastError(); continue; }
            HIPCHK(hipEventRecord(e0, h->stream));
            for (int r = 0; r < reps; ++r)
                HIPCHK(h->mixed ? launch_local_solve<float2>(h, (const float2 *)h->d_g, (float2 *)h->d_ring[0], nrhs)
                                : launch_local_solve<double2>(h, (const double2 *)h->d_g, (double2 *)h->d_ring[0], nrhs));
            HIPCHK(hipEventRecord(e1, h->stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (check_abort(h) != DDM_OK) continue;
            double mean = ms / reps;
            if (times_ms) times_ms[v] = mean;
            if (best < 0 || mean < best_ms) { best = v; best_ms = mean; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } catch (const HipFail &e) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        int r = hip_fail(h, e);
        (void)select_variant(h, keep);
        return r;
    }
    return select_variant(h, best >= 0 ? best : keep);
}

// ---------------------------------------------------------------------------
// Continuous batching over slots.  The ring phase follows the handle's global
// step counter; a slot that joins at global step S has its ring entries
// zeroed (no lagged sources) and gets f restricted to the cores as its first
// source, so its k-th own step computes exactly what step k of a solve alone
// computes.  Mixed precision keeps the residual-corrected sources (the slot's
// residual row starts as f).
// ---------------------------------------------------------------------------
}  // extern "C"

static int slots_init(ddm_handle *h) {
    if (!h->slot_steps.empty()) return DDM_OK;
    const Plan &P = h->plan;
    const size_t vb = (size_t)h->nrhs_max * P.nglob * sizeof(double2);
    HIPCHK(launch_fill_zero(h->d_fin, (long long)vb, h->stream));
    HIPCHK(launch_fill_zero(h->d_uin, (long long)vb, h->stream));
    HIPCHK(launch_fill_zero(h->d_r, (long long)vb, h->stream));
    const size_t es = elem_size(h->mixed);
    HIPCHK(launch_fill_zero(h->d_g, (long long)h->nrhs_max * P.etot * es, h->stream));
    h->g_clean_rows = 0;
    for (int k = 0; k < P.ring; ++k)
        HIPCHK(launch_fill_zero(h->d_ring[k], (long long)h->nrhs_max * P.etot * es, h->stream));
    h->slot_steps.assign(h->nrhs_max, -1);
    h->slot_global = 0;
    std::vector<int> zero(h->nrhs_max, 0);
    set_active(h, zero);
    return DDM_OK;
}

extern "C" int ddm_slot_admit(ddm_handle *h, int slot, const void *f) {
    if (!h || !f || slot < 0 || slot >= h->nrhs_max) return DDM_EINVAL;
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_slot_admit before ddm_factor");
    const Plan &P = h->plan;
    try {
        int st = slots_init(h);
        if (st) return st;
        if (h->slot_steps[slot] >= 0) return fail(h, DDM_EINVAL, "slot in use");
        const size_t vb = (size_t)P.nglob * sizeof(double2);
        const size_t es = elem_size(h->mixed);
        HIPCHK(hipMemcpyAsync(h->d_fin + (size_t)slot * P.nglob, f, vb, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->d_r + (size_t)slot * P.nglob, f, vb, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(launch_fill_zero(h->d_uin + (size_t)slot * P.nglob, (long long)vb, h->stream));
        for (int k = 0; k < P.ring; ++k)
            HIPCHK(launch_fill_zero((char *)h->d_ring[k] + (size_t)slot * P.etot * es, (long long)P.etot * es,
                                    h->stream));
        h->slot_steps[slot] = 0;
        int one = 1;
        HIPCHK(hipMemcpyAsync(h->d_active + slot, &one, sizeof(int), hipMemcpyHostToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

template <typename T>
static void slots_step_impl(ddm_handle *h, int nsteps) {
    const Plan &P = h->plan;
    // slots past the highest busy one are left alone: a slot's arithmetic
    // does not depend on the others, and a slot's state is cleared when it
    // is admitted.  The source norms stay at offset nrhs_max of d_norm, where
    // ddm_slots_poll reads them.
    int n = 0;
    for (int q = 0; q < h->nrhs_max; ++q)
        if (h->slot_steps[q] >= 0) n = q + 1;
    if (n == 0) return;
    const size_t es = sizeof(T);
    const double2 *rcorr = h->mixed ? h->d_r : nullptr;
    for (int k = 0; k < nsteps; ++k) {
        const long long s = ++h->slot_global;
        T *g = (T *)h->d_g;
        HIPCHK((launch_transfer<T, T>(h, ring_at<T>(h, (int)(s - 1)), ring_at<T>(h, (int)(s - 2)),
                                      ring_at<T>(h, (int)(s - 3)), g, n, rcorr)));
        // slots at their first step: f restricted to the cores
        for (int q = 0; q < n; ++q)
            if (h->slot_steps[q] == 0)
                HIPCHK((launch_restrict<double2, T>(h, h->d_fin + (size_t)q * P.nglob, g + (size_t)q * P.etot, 1)));
        T *us = (T *)h->d_ring[s % P.ring];
        HIPCHK(launch_local_solve<T>(h, g, us, n));
        HIPCHK(launch_assemble<T>(h, us, h->d_uin, n, true, h->d_active));
        HIPCHK(launch_residual(h, h->d_fin, h->d_uin, const_cast<double2 *>(rcorr), n, h->d_norm,
                               h->d_norm + h->nrhs_max));
        for (int q = 0; q < n; ++q)
            if (h->slot_steps[q] >= 0) ++h->slot_steps[q];
    }
    (void)es;
}

extern "C" {

int ddm_slots_step(ddm_handle *h, int nsteps) {
    if (!h || nsteps < 0) return DDM_EINVAL;
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_slots_step before ddm_factor");
    try {
        int st = slots_init(h);
        if (st) return st;
        if (h->mixed) slots_step_impl<float2>(h, nsteps);
        else slots_step_impl<double2>(h, nsteps);
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

int ddm_slots_poll(ddm_handle *h, double *relres, int *steps) {
    if (!h) return DDM_EINVAL;
    const int n = h->nrhs_max;
    try {
        int st = slots_init(h);
        if (st) return st;
        std::vector<double> rel;
        fetch_norms(h, n, rel);
        for (int q = 0; q < n; ++q) {
            bool occ = h->slot_steps[q] >= 0;
            if (relres) relres[q] = occ && h->slot_steps[q] > 0 ? rel[q] : -1.0;
            if (steps) steps[q] = h->slot_steps[q];
        }
        return check_abort(h);
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
}

int ddm_slot_retire(ddm_handle *h, int slot, void *u) {
    if (!h || slot < 0 || slot >= h->nrhs_max) return DDM_EINVAL;
    const Plan &P = h->plan;
    try {
        int st = slots_init(h);
        if (st) return st;
        if (h->slot_steps[slot] < 0) return fail(h, DDM_EINVAL, "slot is free");
        if (u)
            HIPCHK(hipMemcpyAsync(u, h->d_uin + (size_t)slot * P.nglob, (size_t)P.nglob * sizeof(double2),
                                  hipMemcpyDeviceToDevice, h->stream));
        int zero = 0;
        HIPCHK(hipMemcpyAsync(h->d_active + slot, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream));
        // a free slot iterates on zero data: clear its source and residual rows
        HIPCHK(launch_fill_zero(h->d_fin + (size_t)slot * P.nglob, (long long)P.nglob * sizeof(double2), h->stream));
        HIPCHK(launch_fill_zero(h->d_r + (size_t)slot * P.nglob, (long long)P.nglob * sizeof(double2), h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        h->slot_steps[slot] = -1;
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

const char *ddm_version(void) { return "libddm 0.1 (gfx950, HIP)"; }

const char *ddm_last_error(const ddm_handle *h) { return h ? h->err.c_str() : g_setup_error.c_str(); }

int ddm_memory_required(const ddm_problem *p, int nrhs_max, size_t *bytes) {
    if (!bytes || nrhs_max < 1) return fail(nullptr, DDM_EINVAL, "bytes must be non-null and nrhs_max >= 1");
    Plan P;
    std::string err;
    int st = build_plan(p, &P, &err);
    if (st) return fail(nullptr, st, err);
    *bytes = plan_bytes(P, p->precision == DDM_MIXED, nrhs_max, 0);
    return DDM_OK;
}

// PML strength for a target reflection R of the quadratic profile
// sigma0 (t/delta)^2: a wave of wave number k crossing the layer twice is
// damped by exp(-2 k int_0^delta sigma) = exp(-2 k sigma0 delta / 3).
static double sigma0_from_reflection(double R, double k_ref, double delta) {
    return 3.0 * std::log(1.0 / R) / (2.0 * k_ref * delta);
}

int ddm_setup(const ddm_problem *p, const double *k2, int nrhs_max, void *stream, ddm_handle **out) {
    if (!out || !k2 || !p || nrhs_max < 1)
        return fail(nullptr, DDM_EINVAL, "p, out and k2 must be non-null, nrhs_max >= 1");
    *out = nullptr;
    ddm_problem pv = *p;
    if (!(pv.reflection >= 0 && pv.reflection < 1))
        return fail(nullptr, DDM_EINVAL, "reflection must lie in [0, 1)");
    if (pv.reflection > 0 && pv.sigma0 != 0)
        return fail(nullptr, DDM_EINVAL, "give sigma0 or reflection, not both");
    std::vector<double> hk2;
    {
        // the grid size, then k2 (host copy: finiteness check, k_ref)
        Plan P0;
        std::string e0;
        ddm_problem pz = pv;
        pz.sigma0 = 0;
        int s0 = build_plan(&pz, &P0, &e0);
        if (s0) return fail(nullptr, s0, e0);
        hk2.resize(P0.nglob);
        if (pv.k2_on_host) {
            memcpy(hk2.data(), k2, P0.nglob * sizeof(double));
        } else if (hipMemcpy(hk2.data(), k2, P0.nglob * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipGetLastError();
            return fail(nullptr, DDM_EINVAL, "k2 could not be read as a device pointer (set k2_on_host for host memory)");
        }
        double kmin2 = INFINITY;
        for (double v : hk2) {
            if (!std::isfinite(v)) return fail(nullptr, DDM_EINVAL, "k2 has non-finite entries");
            kmin2 = std::min(kmin2, v);
        }
        if (pv.reflection > 0) {
            if (!(kmin2 > 0)) return fail(nullptr, DDM_EINVAL, "reflection needs k2 > 0 everywhere (k_ref = sqrt(min k2))");
            pv.sigma0 = sigma0_from_reflection(pv.reflection, std::sqrt(kmin2), pv.n_pml * pv.h);
        }
    }
    ddm_handle *h = new (std::nothrow) ddm_handle();
    if (!h) return fail(nullptr, DDM_ENOMEM, "host allocation failed");
    std::string err;
    int st = build_plan(&pv, &h->plan, &err);
    if (st) { delete h; return fail(nullptr, st, err); }
    {
        // the chain launches need every workgroup resident: bound them by this
        // device's compute units (the plan assumes 256 until it knows)
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0) {
            h->plan.ncu = ncu;
            if (h->plan.twisted && !plan_twist_fits(h->plan)) plan_set_twist(&h->plan, false);
        }
        h->device = dev;
    }
    h->prob = pv;
    h->mixed = p->precision == DDM_MIXED;
    h->nrhs_max = nrhs_max;
    h->stream = (hipStream_t)stream;
    const Plan &P = h->plan;
    size_t need = plan_bytes(P, h->mixed, nrhs_max, 0);
    if (p->hbm_budget_bytes > 0 && need > p->hbm_budget_bytes) {
        char buf[160];
        snprintf(buf, sizeof buf, "plan needs %zu bytes, budget is %zu", need, p->hbm_budget_bytes);
        delete h;
        return fail(nullptr, DDM_ENOMEM, buf);
    }
    {
        // the static scratch of the allocation-free entry points: its device
        // address on this device, looked up once
        hipError_t se = scratch_init(h->device);
        if (se != hipSuccess) {
            char buf[160];
            snprintf(buf, sizeof buf, "static scratch lookup failed on device %d: %s", h->device,
                     hipGetErrorString(se));
            delete h;
            return fail(nullptr, DDM_EHIP, buf);
        }
    }
    try {
        dalloc(h, &h->d_subs, P.subs.size());
        dalloc(h, &h->d_coef, P.coef.size());
        dalloc(h, &h->d_gcoef, P.gcoef.size());
        dalloc(h, &h->d_aown, P.aown.size());
        dalloc(h, &h->d_strip, P.strip.size() > 0 ? P.strip.size() : 1);
        dalloc(h, &h->d_btab, P.btab.size());
        dalloc(h, &h->d_items, P.items.size());
        dalloc(h, &h->d_k2, (size_t)P.nglob);
        dalloc(h, &h->d_flags, (size_t)3 * P.nsub);
        HIPCHK(hipMemcpy(h->d_subs, P.subs.data(), P.subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(h->d_coef, P.coef.data(), P.coef.size() * sizeof(Coef), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(h->d_gcoef, P.gcoef.data(), P.gcoef.size() * sizeof(Coef), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(h->d_aown, P.aown.data(), P.aown.size() * sizeof(AxisOwn), hipMemcpyHostToDevice));
        if (!P.strip.empty())
            HIPCHK(hipMemcpy(h->d_strip, P.strip.data(), P.strip.size() * sizeof(int2), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(h->d_btab, P.btab.data(), P.btab.size() * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(h->d_items, P.items.data(), P.items.size() * sizeof(SolveItem), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(h->d_k2, hk2.data(), P.nglob * sizeof(double), hipMemcpyHostToDevice));
        size_t es = elem_size(h->mixed);
        dalloc(h, (char **)&h->d_W, (size_t)P.fel * es);
        dalloc(h, (char **)&h->d_g, (size_t)nrhs_max * P.etot * es);
        for (int k = 0; k < P.ring; ++k) dalloc(h, (char **)&h->d_ring[k], (size_t)nrhs_max * P.etot * es);
        dalloc(h, &h->d_r, (size_t)nrhs_max * P.nglob);
        if (h->mixed) dalloc(h, &h->d_wide, (size_t)nrhs_max * P.etot);
        h->part_cap = part_doubles(P, nrhs_max, 30);
        dalloc(h, &h->d_part, h->part_cap);
        dalloc(h, &h->d_norm, (size_t)4 * nrhs_max);
        dalloc(h, &h->d_active, (size_t)nrhs_max);
        h->sync_tiles = sync_tiles_for(nrhs_max);
        dalloc(h, &h->d_sync, (size_t)4 * P.nsub * h->sync_tiles + 1);
        HIPCHK(hipMemset(h->d_sync, 0, ((size_t)4 * P.nsub * h->sync_tiles + 1) * sizeof(int)));
        if (chain2_fits(P)) {
            dalloc(h, &h->d_sync2, (size_t)12 * P.nsub);
            dalloc(h, (char **)&h->d_xbuf, chain2_xbuf_bytes(P));
        }
        dalloc(h, &h->d_fin, (size_t)nrhs_max * P.nglob);
        dalloc(h, &h->d_uin, (size_t)nrhs_max * P.nglob);
        if (h->bytes != setup_bytes(P, h->mixed, nrhs_max)) {
            char buf[160];
            snprintf(buf, sizeof buf, "internal: setup allocated %zu bytes, the plan counts %zu", h->bytes,
                     setup_bytes(P, h->mixed, nrhs_max));
            free_all(h);
            delete h;
            return fail(nullptr, DDM_EHIP, buf);
        }
        h->solve_variant = default_variant(h);
        h->plan.mma = h->solve_variant == kSolveMma;
        HIPCHK(hipHostMalloc((void **)&h->h_norm, 4 * nrhs_max * sizeof(double), hipHostMallocDefault));
        std::vector<int> ones(nrhs_max, 1);
        HIPCHK(hipMemcpy(h->d_active, ones.data(), nrhs_max * sizeof(int), hipMemcpyHostToDevice));
    } catch (const HipFail &e) {
        int code = hip_fail(nullptr, e);
        free_all(h);
        delete h;
        return code;
    }
    *out = h;
    return DDM_OK;
}

void ddm_destroy(ddm_handle *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    free_all(h);
    delete h;
}

int ddm_pml_strength(const ddm_handle *h, double *sigma0) {
    if (!h || !sigma0) return DDM_EINVAL;
    *sigma0 = h->plan.sigma0;
    return DDM_OK;
}

int ddm_device_bytes(const ddm_handle *h, size_t *held, size_t *peak) {
    if (!h) return DDM_EINVAL;
    if (held) *held = h->bytes;
    if (peak) *peak = h->peak_bytes;
    return DDM_OK;
}

int ddm_sizes(const ddm_handle *h, long *out) {
    if (!h || !out) return DDM_EINVAL;
    out[0] = (long)h->plan.nglob;
    out[1] = (long)h->plan.etot;
    out[2] = h->plan.nsub;
    out[3] = (long)(h->plan.fel * elem_size(h->mixed));
    return DDM_OK;
}

int ddm_geometry(const ddm_handle *h, int a, long *out) {
    if (!h || !out || a < 0 || a >= h->plan.nsub) return DDM_EINVAL;
    const SubDesc &s = h->plan.subs[a];
    for (int d = 0; d < 3; ++d) {
        out[d] = s.clo[d];
        out[3 + d] = s.chi[d];
        out[6 + d] = s.lo[d];
        out[9 + d] = s.hi[d];
    }
    out[12] = (long)s.off;
    out[13] = (long)s.nloc;
    return DDM_OK;
}

int ddm_factor(ddm_handle *h) {
    if (!h) return DDM_EINVAL;
    const Plan &P = h->plan;
    try {
        if (!h->d_scratch) dalloc(h, (char **)&h->d_scratch, factor_ws_bytes(P));
        if (h->mixed) HIPCHK(launch_factor<float2>(h, h->d_scratch));
        else HIPCHK(launch_factor<double2>(h, h->d_scratch));
        std::vector<int> flags(3 * P.nsub);
        HIPCHK(hipMemcpyAsync(flags.data(), h->d_flags, 3 * P.nsub * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        dfree(h, (char **)&h->d_scratch, factor_ws_bytes(P));
        for (int q = 0; q < 3 * P.nsub; ++q)
            if (flags[q]) {
                char buf[160];
                int a = q < 2 * P.nsub ? q / 2 : q - 2 * P.nsub;
                int t = flags[q] - 1;
                snprintf(buf, sizeof buf, "subdomain %d: pivot below threshold in block %d, column %d", a,
                         t / P.subs[a].bs, t % P.subs[a].bs);
                h->factored = false;
                return fail(h, DDM_ESINGULAR, buf);
            }
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    h->factored = true;
    return DDM_OK;
}

int ddm_apply(ddm_handle *h, const void *u, void *out, int nrhs) {
    int st = check_args(h, nrhs);
    if (st) return st;
    try {
        HIPCHK(launch_apply(h, (const double2 *)u, (double2 *)out, nrhs));
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

int ddm_residual(ddm_handle *h, const void *f, const void *u, void *r, int nrhs, double *rnorm2, double *fnorm2) {
    int st = check_args(h, nrhs);
    if (st) return st;
    try {
        HIPCHK(launch_residual(h, (const double2 *)f, (const double2 *)u, (double2 *)r, nrhs, h->d_norm,
                               h->d_norm + nrhs));
        HIPCHK(hipMemcpyAsync(h->h_norm, h->d_norm, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int q = 0; q < nrhs; ++q) {
            if (rnorm2) rnorm2[q] = h->h_norm[q];
            if (fnorm2) fnorm2[q] = h->h_norm[nrhs + q];
        }
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

int ddm_restrict_core(ddm_handle *h, const void *f, void *g, int nrhs) {
    int st = check_args(h, nrhs);
    if (st) return st;
    try {
        HIPCHK((launch_restrict<double2, double2>(h, (const double2 *)f, (double2 *)g, nrhs)));
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

int ddm_transfer(ddm_handle *h, const void *lag1, const void *lag2, const void *lag3, void *g, int nrhs) {
    int st = check_args(h, nrhs);
    if (st) return st;
    try {
        HIPCHK((launch_transfer<double2, double2>(h, (const double2 *)lag1, (const double2 *)lag2,
                                                  (const double2 *)lag3, (double2 *)g, nrhs)));
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

int ddm_assemble(ddm_handle *h, const void *U, void *u, int nrhs) {
    int st = check_args(h, nrhs);
    if (st) return st;
    try {
        HIPCHK(launch_assemble<double2>(h, (const double2 *)U, (double2 *)u, nrhs, false, nullptr));
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
    return DDM_OK;
}

int ddm_local_solve(ddm_handle *h, const void *g, void *uhat, int nrhs) {
    int st = check_args(h, nrhs);
    if (st) return st;
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_local_solve before ddm_factor");
    const Plan &P = h->plan;
    long long n = (long long)nrhs * P.etot;
    try {
        if (h->mixed) {
            h->g_clean_rows = 0;
            HIPCHK(launch_convert_c128_to_c64((const double2 *)g, (float2 *)h->d_g, n, h->stream));
            HIPCHK(launch_local_solve<float2>(h, (const float2 *)h->d_g, (float2 *)h->d_ring[0], nrhs));
            HIPCHK(launch_convert_c64_to_c128((const float2 *)h->d_ring[0], (double2 *)uhat, n, h->stream));
        } else {
            const double2 *src = (const double2 *)g;
            if (g == uhat) {
                h->g_clean_rows = 0;
                HIPCHK(hipMemcpyAsync(h->d_g, g, n * sizeof(double2), hipMemcpyDeviceToDevice, h->stream));
                src = (const double2 *)h->d_g;
            }
            HIPCHK(launch_local_solve<double2>(h, src, (double2 *)uhat, nrhs));
        }
        return check_abort(h);
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
}

int ddm_iterate(ddm_handle *h, const void *f, void *u, int nrhs, int nsteps, double *relres) {
    int st = check_args(h, nrhs);
    if (st) return st;
    if (slots_busy(h)) return fail(h, DDM_ESTATE, "slots are in use: retire them before a batch solve");
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_iterate before ddm_factor");
    if (nsteps < 0) return fail(h, DDM_EINVAL, "nsteps < 0");
    const Plan &P = h->plan;
    try {
        HIPCHK(launch_fill_zero(u, (long long)nrhs * P.nglob * sizeof(double2), h->stream));
        std::vector<int> ones(nrhs, 1);
        set_active(h, ones);
        std::vector<double> rel;
        auto check = [&](int it, const double2 **) -> bool {
            if (relres) {
                fetch_norms(h, nrhs, rel);
                for (int q = 0; q < nrhs; ++q) relres[(size_t)(it - 1) * nrhs + q] = rel[q];
            }
            return true;
        };
        if (h->mixed) run_steps<float2>(h, (const double2 *)f, (double2 *)u, nrhs, nsteps, check);
        else run_steps<double2>(h, (const double2 *)f, (double2 *)u, nrhs, nsteps, check);
        return check_abort(h);
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    }
}

int ddm_solve(ddm_handle *h, const void *f, void *u, int nrhs, const ddm_solve_opts *opts, ddm_rhs_info *info) {
    int st = check_args(h, nrhs);
    if (st) return st;
    if (slots_busy(h)) return fail(h, DDM_ESTATE, "slots are in use: retire them before a batch solve");
    if (!opts) return fail(h, DDM_EINVAL, "opts is null");
    if (!h->factored) return fail(h, DDM_ESTATE, "ddm_solve before ddm_factor");
    if (!(opts->tol > 0) || opts->maxiter < 1) return fail(h, DDM_EINVAL, "tol must be > 0 and maxiter >= 1");
    try {
        // reject non-finite sources up front
        std::vector<double> rel, fn;
        HIPCHK(launch_norm2(h, (const double2 *)f, h->plan.nglob, nrhs, h->plan.nglob, h->d_norm + 2 * nrhs));
        HIPCHK(hipMemcpyAsync(h->h_norm, h->d_norm + 2 * nrhs, nrhs * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        for (int q = 0; q < nrhs; ++q)
            if (!std::isfinite(h->h_norm[q])) return fail(h, DDM_EINVAL, "source has non-finite entries");
        ddm_solve_opts o = *opts;
        int r;
        if (o.method == DDM_FGMRES)
            r = h->mixed ? solve_fgmres<float2>(h, (const double2 *)f, (double2 *)u, nrhs, o, info)
                         : solve_fgmres<double2>(h, (const double2 *)f, (double2 *)u, nrhs, o, info);
        else
            r = h->mixed ? solve_stationary<float2>(h, (const double2 *)f, (double2 *)u, nrhs, o, info)
                         : solve_stationary<double2>(h, (const double2 *)f, (double2 *)u, nrhs, o, info);
        int a = check_abort(h);
        return a != DDM_OK ? a : r;
    } catch (const HipFail &e) {
        return hip_fail(h, e);
    } catch (const std::string &s) {
        return fail(h, DDM_EINVAL, s);
    }
}

}  // extern "C"
