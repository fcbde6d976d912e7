// Restarted (flexible) GMRES driver with FP64 iterative refinement, for one
// array or a batch of arrays of different shapes (Sec. III-C; right-hand sides
// are the element-port excitations of Sec. IV).
//
// Outer loop (FP64): r = V - Z x with the FP64 MLFFT product; every column whose
// true relative residual ||r_w|| / ||V_w|| is above tol gets an inner solve of
// Z d = r_w / ||r_w|| in the inner precision, and x_w += ||r_w|| d_w.
// Inner solve: per-column restarted GMRES(m), right preconditioned (flexible
// when the preconditioner is the learned correction), classical Gram-Schmidt
// with re-orthogonalisation and FP64 accumulation, Givens least squares in FP64
// and per-column retirement once the residual estimate meets the column's
// target.  With the FP64 inner precision this is plain FP64 GMRES; the outer
// loop then only confirms the true residual.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "krylov.h"
#include "lib.h"

using namespace mlfft;

// most Krylov steps one captured graph may hold (use_graph)
static const int kMaxGraphSteps = 8;

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return c->hip_fail(e_, what);  \
    } while (0)
#define STCHK(call)                                          \
    do {                                                     \
        mlfft_status s_ = (call);                            \
        if (s_ < 0) return s_;                               \
    } while (0)

namespace {

struct Seg {           // one array of the batch
    Array* arr;
    int W;
    size_t off;        // first element of the array's columns inside a batch vector
    size_t N;          // unknowns per column
    const void* V;     // caller's excitations (complex128)
    void* I;           // caller's solution (complex128)
};

// Device memory for one solve, carved out of the context's solve workspaces.
struct Work {
    size_t S = 0;                 // elements of one batch vector
    int Wt = 0;                   // total columns
    size_t maxN = 0;
    // FP64 vectors
    double2 *v64, *x64, *r64;
    // inner-precision vectors (bytes eb per element)
    void *rT, *dT, *tmpT, *tmp2T, *Vb, *Zb;
    // per column
    size_t* coff;
    int* cN;
    double *vnorm, *rnorm, *target, *est, *hist;
    const double* kscale;         // norm of each Krylov column's unscaled right-hand side
    const int* seg_of = nullptr;  // host: array (segment) of each column, per-RHS mode only
    const int* colN = nullptr;    // host: entries of each column
    bool zstore = false;          // Zb holds the preconditioned directions
    int *state, *kcyc, *iters, *mask;
    double2 *H, *g, *sn, *y;
    double* cs;
};

}  // namespace

static size_t align_up(size_t v) { return (v + 255) / 256 * 256; }

mlfft_status solve_impl(Ctx* c, std::vector<Seg>& segs, const mlfft_solve_opts& o, mlfft_solve_info* info);

extern "C" mlfft_status mlfft_solve_default_opts(mlfft_solve_opts* o) {
    if (!o) return MLFFT_E_ARG;
    o->restart = 30;
    o->max_restarts = 100;
    o->tol = 1e-6;
    o->inner_prec = MLFFT_FP32;
    o->inner_tol = 0.0;     // automatic: the accuracy floor of the inner precision
    o->max_outer = 10;
    o->precond = 1;
    o->orth = 2;
    o->x0_given = 0;
    o->record_history = 0;
    o->use_graph = 0;
    o->mode = 0;
    o->pc_bf16 = 0;
    return MLFFT_OK;
}

static mlfft_status check_opts(Ctx* c, const mlfft_solve_opts& o) {
    if (o.restart < 1 || o.restart > 31) return c->fail(MLFFT_E_ARG, "restart must be in [1, 31]");
    if (o.max_restarts < 1) return c->fail(MLFFT_E_ARG, "max_restarts must be >= 1");
    if (!(o.tol > 0.0) || !(o.tol < 1.0)) return c->fail(MLFFT_E_ARG, "tol must be in (0, 1)");
    if (o.inner_prec < MLFFT_FP64 || o.inner_prec > MLFFT_FP32_BF16GEMM)
        return c->fail(MLFFT_E_ARG, "invalid inner precision");
    if (o.inner_prec != MLFFT_FP64 && (!(o.inner_tol >= 0.0) || !(o.inner_tol < 1.0)))
        return c->fail(MLFFT_E_ARG, "inner_tol must be in [0, 1)");
    if (o.max_outer < 1) return c->fail(MLFFT_E_ARG, "max_outer must be >= 1");
    if (o.precond < 0 || o.precond > 4) return c->fail(MLFFT_E_ARG, "precond must be 0, 1, 2, 3 or 4");
    if (o.orth != 1 && o.orth != 2) return c->fail(MLFFT_E_ARG, "orth must be 1 or 2");
    if (o.use_graph < 0 || o.use_graph > kMaxGraphSteps)
        return c->fail(MLFFT_E_ARG, "use_graph must be in [0, %d]", kMaxGraphSteps);
    if (o.mode != 0 && o.mode != 1) return c->fail(MLFFT_E_ARG, "mode must be 0 (per right-hand side) or 1 (global)");
    if (o.pc_bf16 != 0 && o.pc_bf16 != 1) return c->fail(MLFFT_E_ARG, "pc_bf16 must be 0 or 1");
    if (o.precond == 3 && !c->net_ready()) return c->fail(MLFFT_E_STATE, "learned preconditioner requested but no network is loaded");
    return MLFFT_OK;
}

// y = alpha * Z x + beta * addend over all segments (x, y, addend are batch vectors)
static mlfft_status batch_matvec(Ctx* c, std::vector<Seg>& segs, const void* x, void* y, const void* addend,
                                 double alpha, double beta, int prec) {
    const int eb = prec_elem_bytes(prec);
    std::vector<MatvecItem> items;
    for (auto& s : segs)
        items.push_back(MatvecItem{s.arr, s.W, (const char*)x + s.off * eb, (char*)y + s.off * eb,
                                   addend ? (const char*)addend + s.off * eb : nullptr, alpha, beta});
    return c->matvec_group(items, prec);
}

// z = P^{-1} r (kind 1 / 2), or the learned correction of the block-circulant output (kind 3)
static mlfft_status batch_precond(Ctx* c, std::vector<Seg>& segs, int kind, const void* r, void* z, void* scratch,
                                  int prec, int* fallbacks, int* net_applies = nullptr, int pc_prec = -1) {
    const int eb = prec_elem_bytes(prec);
    std::vector<MatvecItem> items;
    void* dst = kind == 3 ? scratch : z;
    for (auto& s : segs)
        items.push_back(MatvecItem{s.arr, s.W, (const char*)r + s.off * eb, (char*)dst + s.off * eb, nullptr, 1.0, 0.0});
    STCHK(c->precond_group(items, kind == 3 ? 1 : kind, pc_prec < 0 ? prec : pc_prec));
    if (kind == 3) {
        for (auto& s : segs) {
            mlfft_status st = c->net_correct(s.arr, s.W, (const char*)scratch + s.off * eb, (char*)z + s.off * eb, prec,
                                             fallbacks);
            if (st < 0) return st;
            if (net_applies) *net_applies += 1;
        }
    }
    return MLFFT_OK;
}


// Launch configuration of one Krylov step: everything its captured kernels and
// copies depend on (the arrays, the column layout, the workspace addresses and
// the options).  Buffers that move bump g_mem_epoch, which drops every graph.
static std::string graph_key(Ctx* c, const std::vector<Seg>& segs, const Work& w, const mlfft_solve_opts& o,
                             int prec, int j, const mlfft_solve_info* info) {
    std::string k;
    auto put = [&k](const void* p, size_t n) { k.append((const char*)p, n); };
    const int hl = (info && o.record_history) ? info->history_len : 0;
    const int ints[] = {j, prec, o.precond, o.orth, o.restart, w.Wt, hl, o.mode, o.pc_bf16, o.use_graph};
    put(ints, sizeof ints);
    const void* ptrs[] = {c->solve_ws.p, c->solve_ws2.p, c->pinned, c->spec_a.p, c->spec_b.p,
                          // the carved workspace (its offsets move with the in-place / staged layout and
                          // with the stored preconditioned directions) and the scale of the Krylov columns'
                          // right-hand sides (||V|| at x = 0, ||r|| afterwards), which the rotations read
                          w.v64, w.x64, w.r64, w.rT, w.dT, w.tmpT, w.tmp2T, w.Vb, w.Zb, w.kscale, w.H, w.g, w.hist};
    put(ptrs, sizeof ptrs);
    const int flags[] = {w.zstore ? 1 : 0};
    put(flags, sizeof flags);
    put(&w.S, sizeof w.S);
    for (const Seg& sg : segs) {
        put(&sg.arr, sizeof sg.arr);
        put(&sg.W, sizeof sg.W);
    }
    return k;
}

// Run one Krylov step through a HIP graph.  The first time a configuration is
// met the step runs eagerly (making every task table and workspace resident);
// the second time it is captured (relaxed mode: no launch is executed while
// capturing), instantiated and launched; afterwards the cached executable
// graph is launched.  The step contains kernels and one device-to-host copy
// into pinned memory, no memset.
template<typename F>
static mlfft_status graph_step(Ctx* c, const std::string& key, F&& step) {
    hipStream_t s = c->stream;
    if (s == nullptr) return step();        // the legacy NULL stream cannot be captured
    if (c->graph_epoch != g_mem_epoch) {
        HIPCHK(hipStreamSynchronize(s), "graph cache");
        c->graphs_release();
        c->graph_epoch = g_mem_epoch;
    }
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        HIPCHK(hipGraphLaunch(it->second, s), "graph launch");
        return MLFFT_OK;
    }
    if (!c->graph_seen.count(key)) {
        c->graph_seen[key] = 1;
        return step();
    }
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "begin capture");
    c->capturing = true;
    const mlfft_status st = step();
    c->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (st < 0 || e != hipSuccess) {
        // nothing was executed while capturing: run the step eagerly instead
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        c->err.clear();
        return step();
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(ei, "graph instantiate");
    HIPCHK(hipGraphLaunch(ex, s), "graph launch");
    if (c->graph_epoch == g_mem_epoch) {
        c->graphs[key] = ex;
    } else {
        HIPCHK(hipStreamSynchronize(s), "graph");
        (void)hipGraphExecDestroy(ex);
    }
    return MLFFT_OK;
}

// The arrays of a batch that still have an iterating column: the batched
// products of a Krylov step skip the others (their columns are retired, and
// the Arnoldi step leaves their slots at zero).  In the global mode there is
// one Krylov column and every array takes part until it retires.
static void active_segs(const std::vector<Seg>& segs, const Work& w, const int* state, int Wk,
                        std::vector<Seg>& act) {
    act.clear();
    if (!w.seg_of || Wk == 1) {
        act = segs;
        return;
    }
    std::vector<char> on(segs.size(), 0);
    for (int i = 0; i < Wk; ++i)
        if (state[i] == 0) on[w.seg_of[i]] = 1;
    for (size_t k = 0; k < segs.size(); ++k)
        if (on[k]) act.push_back(segs[k]);
}

template<typename C>
static mlfft_status inner_solve(Ctx* c, std::vector<Seg>& segs, Work& w, const Cols& cols, const mlfft_solve_opts& o,
                                int prec, mlfft_solve_info* info, std::vector<int>& hstate) {
    hipStream_t s = c->stream;
    const int m = o.restart;
    const int eb = prec_elem_bytes(prec);
    const size_t vb = w.S * eb;
    const bool flexible = o.precond == 3;
    // product precision of the preconditioner inside the Krylov steps: bf16 only
    // when the solution is formed from the stored preconditioned directions
    const int pc_prec = (o.pc_bf16 && prec == P32 && o.precond && w.zstore) ? PBF16 : prec;
    const int Wt = cols.W;      // Krylov columns (1 in the global mode)
    int* pinned_state = c->pinned_state(Wt);
    if (!pinned_state) return c->fail(MLFFT_E_NOMEM, "pinned host buffer");
    // d starts at zero: the first cycle's combination writes it instead of
    // adding to it (d_written), and d is cleared only if no cycle ran
    bool d_written = false;
    HIPCHK(hipMemsetAsync(w.kcyc, 0, Wt * sizeof(int), s), "zero k");
    for (int cyc = 0; cyc < o.max_restarts; ++cyc) {
        const void* res = w.rT;
        if (cyc > 0) {
            STCHK(batch_matvec(c, segs, w.dT, w.tmpT, w.rT, -1.0, 1.0, prec));
            if (info) info->matvecs_inner += 1;
            res = w.tmpT;
        }
        HIPCHK(k_cycle_start<C>(res, w.Vb, cols, w.g, m, w.state, w.target, w.kcyc, w.est, s), "cycle start");
        HIPCHK(hipMemcpyAsync(pinned_state, w.state, Wt * sizeof(int), hipMemcpyDeviceToHost, s), "state");
        HIPCHK(hipStreamSynchronize(s), "cycle start");
        int running = 0;
        for (int i = 0; i < Wt; ++i) running += pinned_state[i] == 0;
        if (running == 0) break;
        std::vector<Seg> act;
        active_segs(segs, w, pinned_state, Wt, act);
        // entries of the iterating columns (for the algorithmic traffic of the profile)
        auto running_elems = [&]() {
            double e = 0.0;
            if (w.colN)
                for (int i = 0; i < Wt; ++i) e += pinned_state[i] == 0 ? (double)w.colN[i] : 0.0;
            return e;
        };
        double run_elems = running_elems();
        int j = 0;          // steps taken in this cycle (no column has more)
        while (j < m) {
            // one Krylov step: z_q = P^{-1} v_q, u = Z z_q, orthogonalise, rotate
            auto step = [&](int q) -> mlfft_status {
                void* vq = (char*)w.Vb + (size_t)q * vb;
                void* vnext = (char*)w.Vb + (size_t)(q + 1) * vb;
                const void* zsrc = vq;
                if (o.precond) {
                    void* zdst = w.zstore ? (char*)w.Zb + (size_t)q * vb : w.tmp2T;
                    STCHK(batch_precond(c, act, o.precond, vq, zdst, w.tmpT, prec, nullptr, nullptr, pc_prec));
                    zsrc = zdst;
                }
                STCHK(batch_matvec(c, act, zsrc, vnext, nullptr, 1.0, 0.0, prec));
                // algorithmic traffic of one step: two passes over the q+2 vectors (the second
                // projection of orth == 2 comes from the Gram matrix) and one write for every
                // iterating column, one write (the zeroed slot) for the others
                const double iter_elems = Wt == 1 ? (double)w.S : run_elems;
                const double bytes = (double)eb * (iter_elems * (2 * (q + 2) + 1) + ((double)w.S - iter_elems));
                const int pr = c->prof_begin(PK_ARNOLDI, prec, bytes, 0);
                HIPCHK(k_arnoldi<C>(w.Vb, q, cols, w.H, m, w.state, o.orth, s), "arnoldi");
                c->prof_end(pr);
                HIPCHK(k_givens(w.H, w.cs, w.sn, w.g, q, m, Wt, w.state, w.target, w.kcyc, w.iters, w.est,
                                o.record_history ? w.hist : nullptr, info ? info->history_len : 0, w.kscale, s),
                       "givens");
                return MLFFT_OK;
            };
            // Eagerly the host checks the column states after every step.  With graphs,
            // use_graph steps form one graph and the host checks once per graph: a
            // column that retires inside it is skipped by the remaining steps (their
            // batched product still spends its work on it).
            const int nstep = o.use_graph ? std::min(o.use_graph, m - j) : 1;
            auto steps = [&]() -> mlfft_status {
                for (int q = j; q < j + nstep; ++q) STCHK(step(q));
                HIPCHK(hipMemcpyAsync(pinned_state, w.state, Wt * sizeof(int), hipMemcpyDeviceToHost, s), "state");
                return MLFFT_OK;
            };
            if (o.use_graph) {
                STCHK(graph_step(c, graph_key(c, act, w, o, prec, j, info), steps));
            } else {
                STCHK(steps());
            }
            if (info) {
                if (o.precond) info->precond_applies += nstep;
                if (flexible) info->net_applies += nstep * (int)act.size();
                info->matvecs_inner += nstep;
            }
            j += nstep;
            HIPCHK(hipStreamSynchronize(s), "iteration");
            running = 0;
            for (int i = 0; i < Wt; ++i) running += pinned_state[i] == 0;
            if (running == 0) break;
            active_segs(segs, w, pinned_state, Wt, act);
            run_elems = running_elems();
        }
        HIPCHK(k_lsq(w.H, w.g, w.y, w.kcyc, m, Wt, s), "least squares");
        const int acc = d_written ? 1 : 0;
        if (w.zstore) {
            HIPCHK(k_combine<C>(w.Zb, cols, w.y, w.kcyc, m, j, w.dT, acc, s), "update");
        } else if (o.precond) {
            HIPCHK(k_combine<C>(w.Vb, cols, w.y, w.kcyc, m, j, w.tmpT, 0, s), "update");
            STCHK(batch_precond(c, segs, o.precond, w.tmpT, d_written ? w.tmp2T : w.dT, nullptr, prec, nullptr));
            if (info) info->precond_applies += 1;
            if (d_written) HIPCHK(k_add_cols<C>(w.dT, w.tmp2T, cols, s), "update");
        } else {
            HIPCHK(k_combine<C>(w.Vb, cols, w.y, w.kcyc, m, j, w.dT, acc, s), "update");
        }
        d_written = true;
        // Every column reached its target by the residual estimate within this
        // cycle: the FP64 true residual of the outer loop judges the result, so
        // no inner restart residual is formed.
        if (running == 0) break;
    }
    if (!d_written) HIPCHK(hipMemsetAsync(w.dT, 0, vb, s), "zero d");
    (void)hstate;
    return MLFFT_OK;
}

mlfft_status solve_impl(Ctx* c, std::vector<Seg>& segs, const mlfft_solve_opts& o, mlfft_solve_info* info) {
    hipStream_t s = c->stream;
    const int prec = o.inner_prec;
    const int eb = prec_elem_bytes(prec);
    const int m = o.restart;
    Work w;
    // column layout
    std::vector<size_t> hoff;
    std::vector<int> hN;
    std::vector<int> seg_of;
    size_t S = 0;
    for (size_t i = 0; i < segs.size(); ++i) {
        Seg& sg = segs[i];
        sg.N = sg.arr->Nt();
        sg.off = S;
        for (int q = 0; q < sg.W; ++q) {
            hoff.push_back(S + (size_t)q * sg.N);
            hN.push_back((int)sg.N);
            seg_of.push_back((int)i);
        }
        S += sg.N * sg.W;
        w.maxN = std::max(w.maxN, sg.N);
    }
    w.S = S;
    w.Wt = (int)hoff.size();
    const int Wt = w.Wt;
    if (Wt == 0) return MLFFT_OK;
    const bool flexible = o.precond == 3;
    // Krylov columns: one per right-hand side, or in the global mode (eq. ZIVvec)
    // a single column made of all right-hand sides, with Frobenius inner products
    const bool global = o.mode == 1;
    if (global && S > (size_t)0x7fffffff) return c->fail(MLFFT_E_ARG, "global mode: more than 2^31-1 unknowns in all");
    const int Wk = global ? 1 : Wt;
    std::vector<size_t> hkoff = global ? std::vector<size_t>{0} : hoff;
    std::vector<int> hkN = global ? std::vector<int>{(int)S} : hN;
    // V and I are used in place (no gather of V, no scatter of x) when the
    // batch's columns already lie back to back in batch order in both and the
    // two ranges do not overlap; otherwise they are copied to and from the
    // workspace.
    bool in_place = true;
    {
        const char* v0 = (const char*)segs[0].V;
        char* i0 = (char*)segs[0].I;
        for (const Seg& sg : segs)
            in_place = in_place && (const char*)sg.V == v0 + sg.off * 16 && (char*)sg.I == i0 + sg.off * 16;
        const bool disjoint = i0 + S * 16 <= v0 || v0 + S * 16 <= (const char*)i0;
        in_place = in_place && disjoint;
    }
    // carve the workspaces
    const size_t v64b = align_up(S * 16), vTb = align_up(S * eb);
    const size_t n64 = in_place ? 1 : 3;                     // FP64 batch vectors in the workspace
    // Preconditioned directions z_j = P^{-1} v_j are kept (m more vectors) when the
    // solve is flexible, and also with a fixed preconditioner when the memory is
    // there: x = Z y then replaces x = P^{-1} (V y), one preconditioner apply less
    // per cycle.  Without the memory the fixed preconditioner is applied to V y.
    const size_t big0 = n64 * v64b + 4 * vTb + (size_t)(m + 1) * vTb;
    const size_t bigz = big0 + (size_t)m * vTb;
    const int hist_len = (info && o.record_history) ? info->history_len : 0;
    // Arnoldi chunks of every column and their partial-sum rows
    std::vector<int> hchoff(Wk + 1, 0);
    for (int i = 0; i < Wk; ++i) hchoff[i + 1] = hchoff[i] + arnoldi_chunks((size_t)hkN[i]);
    const int nch = hchoff[Wk];
    const size_t partb = align_up((size_t)nch * (4 * m + 3) * sizeof(double));
    const size_t hsb = align_up((size_t)Wk * (4 * m + 3) * sizeof(double));
    const size_t gramb = o.orth == 2 ? align_up((size_t)Wk * (m + 1) * (m + 1) * 16) : 0;
    size_t small = align_up((Wt + 1) * sizeof(int)) + partb + hsb + gramb + align_up(sizeof(size_t)) + align_up(sizeof(int)) +
                   align_up(Wt * sizeof(double)) + align_up(Wt * sizeof(size_t)) + 5 * align_up(Wt * sizeof(int)) +
                   6 * align_up(Wt * sizeof(double)) + align_up((size_t)Wt * (m + 1) * m * 16) +
                   align_up((size_t)Wt * (m + 1) * 16) + 2 * align_up((size_t)Wt * m * 16) +
                   align_up((size_t)Wt * m * 8) + align_up((size_t)std::max(hist_len, 1) * Wt * 8);
    bool zstore = flexible;
    if (flexible) {
        HIPCHK(c->solve_ws.ensure(bigz), "Krylov workspace");
    } else if (o.precond && c->solve_ws.ensure(bigz) == hipSuccess) {
        zstore = true;
    } else {
        (void)hipGetLastError();
        HIPCHK(c->solve_ws.ensure(big0), "Krylov workspace");
    }
    w.zstore = zstore;
    HIPCHK(c->solve_ws2.ensure(small), "Krylov workspace");
    // The spectral workspaces of the largest product of the solve (the FP64 true
    // residual of every array) are reserved here as well, so that a solve too large
    // for the device fails with MLFFT_E_NOMEM before anything is enqueued.
    {
        size_t need = 0;
        for (const Seg& sg : segs) {
            need += (size_t)sg.arr->K * sg.arr->b * sg.W * 16;
            need = align_up(need);
        }
        HIPCHK(c->spec_a.ensure(need), "spectral workspace");
        HIPCHK(c->spec_b.ensure(need), "spectral workspace");
    }
    char* p = (char*)c->solve_ws.p;
    if (in_place) {
        w.v64 = (double2*)const_cast<void*>(segs[0].V);    // read only
        w.x64 = (double2*)segs[0].I;
    } else {
        w.v64 = (double2*)p; p += v64b;
        w.x64 = (double2*)p; p += v64b;
    }
    w.r64 = (double2*)p; p += v64b;
    w.rT = p; p += vTb;
    w.dT = p; p += vTb;
    w.tmpT = p; p += vTb;
    w.tmp2T = p; p += vTb;
    w.Vb = p; p += (size_t)(m + 1) * vTb;
    w.Zb = zstore ? (void*)p : nullptr;
    char* q = (char*)c->solve_ws2.p;
    int* choff = (int*)q; q += align_up((Wt + 1) * sizeof(int));
    double* part1 = (double*)q; q += partb;
    double* hsum1 = (double*)q; q += hsb;
    double2* gram = gramb ? (double2*)q : nullptr; q += gramb;
    size_t* gkoff = (size_t*)q; q += align_up(sizeof(size_t));
    int* gkN = (int*)q; q += align_up(sizeof(int));
    double* gscale = (double*)q; q += align_up(Wt * sizeof(double));
    w.coff = (size_t*)q; q += align_up(Wt * sizeof(size_t));
    w.cN = (int*)q; q += align_up(Wt * sizeof(int));
    w.state = (int*)q; q += align_up(Wt * sizeof(int));
    w.kcyc = (int*)q; q += align_up(Wt * sizeof(int));
    w.iters = (int*)q; q += align_up(Wt * sizeof(int));
    w.mask = (int*)q; q += align_up(Wt * sizeof(int));
    w.vnorm = (double*)q; q += align_up(Wt * sizeof(double));
    w.rnorm = (double*)q; q += align_up(Wt * sizeof(double));
    w.target = (double*)q; q += align_up(Wt * sizeof(double));
    w.est = (double*)q; q += align_up(Wt * sizeof(double));
    double* scratch_d = (double*)q; q += align_up(Wt * sizeof(double));
    q += align_up(Wt * sizeof(double));
    w.H = (double2*)q; q += align_up((size_t)Wt * (m + 1) * m * 16);
    w.g = (double2*)q; q += align_up((size_t)Wt * (m + 1) * 16);
    w.sn = (double2*)q; q += align_up((size_t)Wt * m * 16);
    w.y = (double2*)q; q += align_up((size_t)Wt * m * 16);
    w.cs = (double*)q; q += align_up((size_t)Wt * m * 8);
    w.hist = (double*)q;
    (void)scratch_d;
    Cols cols{w.coff, w.cN, Wt, S, w.maxN};
    Cols kc = global ? Cols{gkoff, gkN, 1, S, S} : cols;
    w.seg_of = global ? nullptr : seg_of.data();
    w.colN = global ? nullptr : hN.data();
    kc.choff = choff;
    kc.nch = nch;
    kc.maxch = 0;
    for (int i = 0; i < Wk; ++i) kc.maxch = std::max(kc.maxch, hchoff[i + 1] - hchoff[i]);
    kc.part1 = part1;
    kc.hsum1 = hsum1;
    kc.gram = gram;
    HIPCHK(hipMemcpyAsync(choff, hchoff.data(), (Wk + 1) * sizeof(int), hipMemcpyHostToDevice, s), "columns");
    if (global) {
        HIPCHK(hipMemcpyAsync(gkoff, hkoff.data(), sizeof(size_t), hipMemcpyHostToDevice, s), "columns");
        HIPCHK(hipMemcpyAsync(gkN, hkN.data(), sizeof(int), hipMemcpyHostToDevice, s), "columns");
    }
    HIPCHK(hipMemcpyAsync(w.coff, hoff.data(), Wt * sizeof(size_t), hipMemcpyHostToDevice, s), "columns");
    HIPCHK(hipMemcpyAsync(w.cN, hN.data(), Wt * sizeof(int), hipMemcpyHostToDevice, s), "columns");
    HIPCHK(hipMemsetAsync(w.iters, 0, Wt * sizeof(int), s), "iters");
    if (hist_len) HIPCHK(hipMemsetAsync(w.hist, 0, (size_t)hist_len * Wt * 8, s), "history");
    // gather V (and x0) into batch vectors.  Without x0, x starts at zero: the
    // first update writes x instead of adding to it (x_written).
    if (!in_place) {
        for (auto& sg : segs) {
            HIPCHK(hipMemcpyAsync(w.v64 + sg.off, sg.V, sg.N * sg.W * 16, hipMemcpyDeviceToDevice, s), "gather V");
            if (o.x0_given)
                HIPCHK(hipMemcpyAsync(w.x64 + sg.off, sg.I, sg.N * sg.W * 16, hipMemcpyDeviceToDevice, s),
                       "gather x0");
        }
    }
    bool x_written = o.x0_given != 0;
    HIPCHK(k_colnorm<double2>(w.v64, cols, w.vnorm, s), "norms");
    std::vector<double> hv(Wt), hr(Wt), ht(Wt);
    std::vector<int> hstate(Wt), outer_used(Wt, 0);
    HIPCHK(hipMemcpyAsync(hv.data(), w.vnorm, Wt * sizeof(double), hipMemcpyDeviceToHost, s), "norms");
    // Accuracy floor of an inner solve.  An FP32 solve can drive the residual
    // estimate to a few 1e-7 of its right-hand side before FP32 rounding of the
    // basis and of the product dominates; the bf16-input block product rounds
    // every transformed vector to 8 significant bits, which makes the inner
    // operator inexact at the 1e-3 level, so its solve is stopped at 1e-2.
    const double inner_floor = o.inner_tol > 0.0 ? o.inner_tol : (prec == PBF16 ? 1e-2 : 3e-7);
    bool r_current = false;     // hr holds the norms of V - Z x64 for the current x64
    bool r_is_v = false;        // the residual of the last step was V itself (x = 0), not stored in r64
    // arrays whose x changed in the last inner solve; in the per-RHS mode the
    // update is masked to the solved columns, so the residual of an array with
    // no solved column is still current
    std::vector<Seg> rsegs = segs;
    // The learned correction is judged by the FP64 true residual: an inner solve asks
    // every column it solves for a reduction of at least 0.3, so a refinement step
    // that leaves the residual of those columns above half of what it was (2-norm
    // over them) means the corrected preconditioner does not work for this system;
    // the remaining steps then use the plain block-circulant preconditioner.
    mlfft_solve_opts oi = o;
    std::vector<double> hprev(Wt, 0.0);
    std::vector<char> solved_prev(Wt, 0);
    for (int outer = 0; outer < o.max_outer; ++outer) {
        const double2* rsrc = w.r64;
        if (outer == 0 && !o.x0_given) {
            // x = 0: the residual is V and its norms are those of V
            rsrc = w.v64;
            r_is_v = true;
            HIPCHK(hipStreamSynchronize(s), "norms");
            hr = hv;
        } else {
            // every array's slot of r64 is recomputed after a step that took the residual from V
            if (r_is_v) rsegs = segs;
            r_is_v = false;
            if (!rsegs.empty()) {
                STCHK(batch_matvec(c, rsegs, w.x64, w.r64, w.v64, -1.0, 1.0, P64));
                if (info) info->matvecs64 += 1;
            }
            HIPCHK(k_colnorm<double2>(w.r64, cols, w.rnorm, s), "norms");
            HIPCHK(hipMemcpyAsync(hr.data(), w.rnorm, Wt * sizeof(double), hipMemcpyDeviceToHost, s), "norms");
            HIPCHK(hipStreamSynchronize(s), "norms");
        }
        if (oi.precond == 3 && outer > 0) {
            double r2 = 0.0, p2 = 0.0;
            for (int i = 0; i < Wt; ++i)
                if (solved_prev[i]) { r2 += hr[i] * hr[i]; p2 += hprev[i] * hprev[i]; }
            if (p2 > 0.0 && r2 > 0.25 * p2) {
                oi.precond = 1;
                if (info) info->pc_switched = 1;
            }
        }
        int active = 0;
        for (int i = 0; i < Wt; ++i) {
            const bool done = !(hv[i] > 0.0) || hr[i] <= o.tol * hv[i];
            if (!std::isfinite(hr[i])) return c->fail(MLFFT_E_ARG, "non-finite residual in column %d (check V and x0)", i);
            hstate[i] = done ? 2 : 0;
            active += !done;
            // inner target, relative to the unit-norm inner right-hand side; an inner
            // solve in reduced precision aims lower, so that its FP64 true residual
            // (estimate plus the inner product's rounding) lands below tol and no
            // second refinement step is needed
            const double need = done ? 1.0 : (prec == P64 ? 0.9 : 0.3) * o.tol * hv[i] / hr[i];
            ht[i] = prec == P64 ? need : std::max(inner_floor, need);
            if (!done) outer_used[i] = outer + 1;
        }
        if (active == 0) { r_current = true; break; }
        if (global) rsegs = segs;
        else active_segs(segs, w, hstate.data(), Wt, rsegs);
        const double* scale = r_is_v ? w.vnorm : w.rnorm;
        if (global) {
            // one inner solve of Z D = R / ||R||_F over all columns.  The first aims at the
            // Frobenius target ||R||_F <= f tol ||V||_F of the vectorised method; once that
            // is met, columns still above their own tol are served by aiming the next solve
            // at ||R||_F <= f tol min ||V_i|| over the unconverged columns, which bounds
            // every column's residual (the Frobenius target would then ask for nothing).
            double v2 = 0.0, r2 = 0.0, vmin = HUGE_VAL;
            for (int i = 0; i < Wt; ++i) {
                v2 += hv[i] * hv[i];
                r2 += hr[i] * hr[i];
                if (hv[i] > 0.0 && hr[i] > o.tol * hv[i]) vmin = std::min(vmin, hv[i]);
            }
            const double f = prec == P64 ? 0.9 : 0.3;
            const bool frob_met = std::sqrt(r2) <= f * o.tol * std::sqrt(v2);
            const double need = frob_met ? f * o.tol * vmin / std::sqrt(r2) : f * o.tol * std::sqrt(v2 / r2);
            ht[0] = prec == P64 ? need : std::max(inner_floor, need);
            hstate[0] = 0;
            std::vector<double> hg(Wt, std::sqrt(r2));
            HIPCHK(hipMemcpyAsync(gscale, hg.data(), Wt * sizeof(double), hipMemcpyHostToDevice, s), "scale");
            HIPCHK(hipStreamSynchronize(s), "scale");
            scale = gscale;
        }
        w.kscale = scale;
        HIPCHK(hipMemcpyAsync(w.state, hstate.data(), Wk * sizeof(int), hipMemcpyHostToDevice, s), "state");
        HIPCHK(hipMemcpyAsync(w.target, ht.data(), Wk * sizeof(double), hipMemcpyHostToDevice, s), "targets");
        HIPCHK(hipStreamSynchronize(s), "state");
        // update mask: the columns that were solved (all of them in the global mode)
        for (int i = 0; i < Wt; ++i) hstate[i] = global ? 1 : hstate[i] == 0;
        HIPCHK(hipMemcpyAsync(w.mask, hstate.data(), Wt * sizeof(int), hipMemcpyHostToDevice, s), "mask");
        if (prec == P64)
            HIPCHK((k_scale_cols<double2, double2>(rsrc, w.rT, cols, scale, 1, s)), "scale r");
        else
            HIPCHK((k_scale_cols<double2, float2>(rsrc, w.rT, cols, scale, 1, s)), "scale r");
        for (int i = 0; i < Wt; ++i) {
            solved_prev[i] = hstate[i] ? 1 : 0;
            hprev[i] = hr[i];
        }
        mlfft_status st = prec == P64 ? inner_solve<double2>(c, segs, w, kc, oi, prec, info, hstate)
                                      : inner_solve<float2>(c, segs, w, kc, oi, prec, info, hstate);
        if (st < 0) return st;
        const int assign = x_written ? 0 : 1;
        if (prec == P64)
            HIPCHK(k_axpy_cols<double2>(w.x64, w.dT, cols, scale, w.mask, assign, s), "update x");
        else
            HIPCHK(k_axpy_cols<float2>(w.x64, w.dT, cols, scale, w.mask, assign, s), "update x");
        x_written = true;
        HIPCHK(hipStreamSynchronize(s), "update x");      // host vectors above are reused next step
    }
    // every column was already converged at x = 0 (zero right-hand sides)
    if (!x_written) HIPCHK(hipMemsetAsync(w.x64, 0, S * 16, s), "zero x");
    // final true FP64 residual (its norms are already at hand when the loop stopped on convergence)
    if (!r_current) {
        STCHK(batch_matvec(c, segs, w.x64, w.r64, w.v64, -1.0, 1.0, P64));
        if (info) info->matvecs64 += 1;
        HIPCHK(k_colnorm<double2>(w.r64, cols, w.rnorm, s), "norms");
        HIPCHK(hipMemcpyAsync(hr.data(), w.rnorm, Wt * sizeof(double), hipMemcpyDeviceToHost, s), "norms");
    }
    std::vector<int> hit(Wk);
    HIPCHK(hipMemcpyAsync(hit.data(), w.iters, Wk * sizeof(int), hipMemcpyDeviceToHost, s), "iters");
    if (!in_place)
        for (auto& sg : segs)
            HIPCHK(hipMemcpyAsync(sg.I, w.x64 + sg.off, sg.N * sg.W * 16, hipMemcpyDeviceToDevice, s), "scatter x");
    std::vector<double> hh;
    if (hist_len) {
        hh.resize((size_t)hist_len * Wk);
        HIPCHK(hipMemcpyAsync(hh.data(), w.hist, hh.size() * 8, hipMemcpyDeviceToHost, s), "history");
    }
    HIPCHK(hipStreamSynchronize(s), "solve");
    if (o.precond == 3 && info) info->fallbacks = c->net_fallbacks_take();
    bool all = true;
    for (int i = 0; i < Wt; ++i) {
        const double rr = hv[i] > 0.0 ? hr[i] / hv[i] : 0.0;
        const bool ok = rr <= o.tol;
        all = all && ok;
        if (info) {
            if (info->relres) info->relres[i] = rr;
            if (info->converged) info->converged[i] = ok;
            if (info->iters) info->iters[i] = hit[global ? 0 : i];
            if (info->outer) info->outer[i] = outer_used[i];
        }
    }
    if (info && info->history && hist_len) {
        // history[it][w]: residual estimate relative to ||V_w|| (global mode: ||R||_F / ||V||_F
        // for every column)
        double v2 = 0.0;
        for (int i = 0; i < Wt; ++i) v2 += hv[i] * hv[i];
        for (int it = 0; it < hist_len; ++it)
            for (int i = 0; i < Wt; ++i) {
                const double e = hh[(size_t)it * Wk + (global ? 0 : i)];
                const double d = global ? std::sqrt(v2) : hv[i];
                info->history[(size_t)it * Wt + i] = d > 0.0 ? e / d : 0.0;
            }
    }
    return all ? MLFFT_OK : MLFFT_NOT_CONVERGED;
}

extern "C" {

mlfft_status mlfft_solve(mlfft_ctx ctx, int array_id, int W, const void* V, void* I, const mlfft_solve_opts* opts,
                         mlfft_solve_info* info) {
    if (!ctx) return MLFFT_E_ARG;
    return mlfft_solve_batch(ctx, 1, &array_id, &W, &V, &I, opts, info);
}

mlfft_status mlfft_solve_batch(mlfft_ctx ctx, int n_arrays, const int* array_ids, const int* Ws,
                               const void* const* V, void* const* I, const mlfft_solve_opts* opts,
                               mlfft_solve_info* info) {
    if (!ctx) return MLFFT_E_ARG;
    Ctx* c = ctx;
    if (n_arrays < 1 || !array_ids || !Ws || !V || !I) return c->fail(MLFFT_E_ARG, "empty or NULL batch description");
    mlfft_solve_opts o;
    if (opts) o = *opts; else mlfft_solve_default_opts(&o);
    STCHK(check_opts(c, o));
    std::vector<Seg> segs;
    for (int i = 0; i < n_arrays; ++i) {
        Array* a = c->find(array_ids[i]);
        if (!a) return c->fail(MLFFT_E_STATE, "unknown array id %d", array_ids[i]);
        for (int j = 0; j < i; ++j)
            if (array_ids[j] == array_ids[i]) return c->fail(MLFFT_E_ARG, "array id %d appears twice", array_ids[i]);
        if (Ws[i] < 0) return c->fail(MLFFT_E_ARG, "W must be >= 0");
        if (o.precond == 3 && a->Nc > 0)
            return c->fail(MLFFT_E_ARG, "the learned correction is not defined for array %d with border unknowns",
                           array_ids[i]);
        if (Ws[i] == 0) continue;
        if (!V[i] || !I[i]) return c->fail(MLFFT_E_ARG, "V or I is NULL for array %d", array_ids[i]);
        segs.push_back(Seg{a, Ws[i], 0, 0, V[i], I[i]});
    }
    if (o.precond == 3) (void)c->net_fallbacks_take();
    if (info) {
        info->fallbacks = 0;
        info->matvecs64 = 0;
        info->matvecs_inner = 0;
        info->precond_applies = 0;
        info->net_applies = 0;
        info->pc_switched = 0;
        if (!info->history) info->history_len = 0;
    }
    HIPCHK(hipSetDevice(c->device), "set device");
    return solve_impl(c, segs, o, info);
}

}  // extern "C"
