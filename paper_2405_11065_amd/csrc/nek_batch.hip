// libnek batches: many independent box problems (each its own mesh and
// order, or many right-hand sides on one mesh) solved together.  Every
// problem keeps a context of its own; problems whose mesh and order repeat
// an earlier problem's share its set-up data (geometric factors, D, mass,
// maps) instead of holding a copy.  A device table per order lets one
// launch of the operator kernel and one of the gather/update kernel advance
// every problem of that order by one CG iteration, each workgroup running
// the solo kernel body on its problem's share; the shares of problems on
// one mesh are interleaved block by block on the same XCD, so that the
// factors one of them streams are still in that XCD's L2 for the others.  A chunk of iterations for all orders (one stream per order, forked
// and joined by events) is recorded once as a HIP graph and replayed; the
// iteration number comes from a device counter the graph advances, so the
// same graph serves every chunk of every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "nek.h"
#include "nek_internal.hpp"

using namespace nek;

namespace nek {
namespace {

struct Group {
    int NP = 0;
    std::vector<int> members;          // problem indices, ascending
    int variant[3] = {0, 0, 0};        // per nek_prec
    BatchProb *dtab = nullptr;         // device table, one entry per member
    BatchProb *htab = nullptr;         // pinned staging of the table
    int2 *downer = nullptr;            // device map workgroup -> (member, block); member -1: none
    long owner_cap = 0;
    int layout_v = -1;                 // variant and members the layout below was built for
    std::vector<char> layout_act;
    unsigned grid = 0;
    std::vector<int> nblk, ngroups;
    bool active = false;               // some member takes part in the current run
    hipStream_t s = nullptr;
    hipEvent_t join = nullptr;
};

}  // namespace
}  // namespace nek

struct nek_batch {
    std::vector<nek_ctx *> ctx;
    std::vector<int> root;             // problem whose set-up data problem i uses (i itself if its own)
    std::vector<int> group_of;
    std::vector<Group> groups;
    hipStream_t stream = nullptr;      // owned; every member context runs on it
    hipStream_t user = nullptr;        // the caller's stream (not owned)
    Scal **dscs = nullptr, **hscs = nullptr;
    Scal *hscal = nullptr;             // pinned read-back of the members' scalars
    int *dbase = nullptr;
    int *hflags = nullptr;             // pinned; [0] = all done, written by k_batch_alldone
    int *dflag = nullptr;              // device alias of hflags (not owned)
    hipEvent_t ev[2] = {nullptr, nullptr}, fork = nullptr, entry = nullptr, t0 = nullptr, t1 = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int> graph_key;
    int64_t chunks = 0, captures = 0;
    int epw_opt = 0;                   // opts.elts_per_wg of the setup
    bool tuned[3] = {false, false, false};
};

namespace nek {
namespace {

int nprob(const nek_batch *b) { return (int)b->ctx.size(); }

// The same mesh: equal element counts and, for a uniform lattice, equal box
// corners, else the same vertex values (an identical pointer or content).
bool same_mesh(const nek_mesh &a, const nek_mesh &b)
{
    for (int d = 0; d < 3; ++d)
        if (a.nel[d] != b.nel[d]) return false;
    if (!a.vtx || !b.vtx) {
        if (a.vtx || b.vtx) return false;
        for (int d = 0; d < 3; ++d)
            if (a.lo[d] != b.lo[d] || a.hi[d] != b.hi[d]) return false;
        return true;
    }
    const size_t nv = 3 * (size_t)(a.nel[0] + 1) * (a.nel[1] + 1) * (a.nel[2] + 1);
    return a.vtx == b.vtx || std::memcmp(a.vtx, b.vtx, nv * sizeof(double)) == 0;
}

// Workgroups of the group's members taking part in a run (act) under
// variant v: each gets exactly the grid of its solo launch; the others get
// none.  The active members on one mesh form a set of K, laid out from a
// multiple of 8: block j of the set's i-th member at
//     8 K floor(j / 8) + 8 i + (j mod 8),
// so block j of every member lands on XCD j mod 8, as in a solo launch, and
// the K blocks that walk the same elements are dispatched together.  Sets
// follow one another in the order of their first member.
int layout(nek_batch *b, Group &G, int v, const std::vector<char> &act)
{
    const size_t n = G.members.size();
    std::vector<char> ga(n);
    for (size_t q = 0; q < n; ++q) ga[q] = act[G.members[q]];
    if (G.layout_v == v && G.layout_act == ga) return NEK_OK;
    const int epw = np_ops(G.NP)->variant_epw(v);
    if (epw <= 0) return NEK_E_ARG;
    G.nblk.assign(n, 0);
    G.ngroups.assign(n, 0);
    std::vector<std::vector<int>> sets;   // member positions q, by mesh
    std::vector<int> set_root;
    for (size_t q = 0; q < n; ++q) {
        const nek_ctx *c = b->ctx[G.members[q]];
        G.ngroups[q] = ax_groups(c, epw);
        if (!ga[q]) continue;
        G.nblk[q] = (int)ax_grid(c, epw, 0);   // batches read stored factors
        const int r = b->root[G.members[q]];
        size_t k = 0;
        while (k < sets.size() && set_root[k] != r) ++k;
        if (k == sets.size()) {
            sets.emplace_back();
            set_root.push_back(r);
        }
        sets[k].push_back((int)q);
    }
    long blk = 0;
    std::vector<std::pair<long, int2>> place;
    for (const auto &S : sets) {
        const long K = (long)S.size(), nb = G.nblk[S[0]];   // one mesh: one grid size
        blk = (blk + 7) / 8 * 8;
        for (long i = 0; i < K; ++i)
            for (long j = 0; j < nb; ++j)
                place.push_back({blk + 8 * K * (j / 8) + 8 * i + (j % 8), make_int2(S[i], (int)j)});
        blk += 8 * K * ((nb + 7) / 8);
    }
    if (blk >= (1L << 31)) return NEK_E_ARG;
    blk = std::max(blk, 1L);
    G.grid = (unsigned)blk;
    std::vector<int2> owner(blk, make_int2(-1, 0));
    for (const auto &pl : place) owner[pl.first] = pl.second;
    if (blk > G.owner_cap) {
        dfree(G.downer);
        if (dalloc(G.downer, blk)) return NEK_E_OOM;
        G.owner_cap = blk;
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemcpy(G.downer, owner.data(), blk * sizeof(int2), hipMemcpyHostToDevice));
    G.layout_v = v;
    G.layout_act = ga;
    return NEK_OK;
}

const void *group_D(const nek_batch *b, const Group &G, int prec)
{
    const nek_ctx *c = b->ctx[G.members[0]];
    return prec == NEK_PREC_FP64 ? (const void *)c->D64 : (const void *)c->D32;
}

// One chunk of CG_CHUNK iterations of every active group, then the all-done
// flag.  Enqueued directly or under capture.
int enqueue_chunk(nek_batch *b, int prec)
{
    int rc;
    const bool x64 = prec != NEK_PREC_FP64 && !b->ctx[0]->opts.corr_fp32;
    if ((rc = batch_advance_launch(b->stream, b->dbase, CHUNK_ITERS))) return rc;
    std::vector<Group *> act;
    for (auto &G : b->groups)
        if (G.active) act.push_back(&G);
    const bool fork = act.size() > 1;
    if (fork) {
        HIP_TRY(hipEventRecord(b->fork, b->stream));
        for (Group *G : act) HIP_TRY(hipStreamWaitEvent(G->s, b->fork, 0));
    }
    for (Group *G : act) {
        const NpOps *o = np_ops(G->NP);
        const hipStream_t s = fork ? G->s : b->stream;
        const void *D = group_D(b, *G, prec);
        for (int q = 1; q <= CHUNK_ITERS; ++q)
            if ((rc = o->batch_iter(s, prec, G->variant[prec], x64, G->dtab, G->downer, G->grid, D, q, b->dbase,
                                    false, false)))
                return rc;
    }
    if (fork)
        for (Group *G : act) {
            HIP_TRY(hipEventRecord(G->join, G->s));
            HIP_TRY(hipStreamWaitEvent(b->stream, G->join, 0));
        }
    return batch_alldone_launch(b->stream, b->dscs, nprob(b), b->dflag);
}

void drop_graph(nek_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_key.clear();
}

int capture_chunk(nek_batch *b, int prec)
{
    drop_graph(b);
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_chunk(b, prec);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess || !g) return NEK_E_HIP;
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        drop_graph(b);
        return NEK_E_HIP;
    }
    ++b->captures;
    return NEK_OK;
}

// CG runs of the problems flagged in act, already started (k_cg_start) on
// their contexts, with iterates xs[m], until every one has stopped (each at
// its own cap) or maxcap iterations are enqueued; then one closing operator
// launch per order.  Synchronises.  With t set, *t = ms from the first chunk
// to the closing launch.
int run_batch(nek_batch *b, int prec, const std::vector<char> &act, const std::vector<void *> &xs, int maxcap,
              bool use_graph, float *t = nullptr)
{
    int rc;
    const int n = nprob(b);
    const bool x64 = prec != NEK_PREC_FP64 && !b->ctx[0]->opts.corr_fp32;
    std::vector<int> key{prec, x64 ? 1 : 0};
    HIP_TRY(hipStreamSynchronize(b->stream));   // staging buffers below are free
    for (auto &G : b->groups) {
        const int v = G.variant[prec];
        if ((rc = layout(b, G, v, act))) return rc;
        G.active = false;
        for (size_t q = 0; q < G.members.size(); ++q) {
            const int m = G.members[q];
            nek_ctx *c = b->ctx[m];
            BatchProb &P = G.htab[q];
            if (prec == NEK_PREC_FP64) {
                P.r = c->r64; P.p = c->p64; P.w = c->w64; P.g = c->g64;
            } else {
                P.r = c->r32; P.p = c->p32; P.w = c->w32;
                P.g = prec == NEK_PREC_BF16G ? (const void *)c->g16 : (const void *)c->g32;
            }
            P.x = xs[m];
            P.sc = c->sc;
            P.partials = c->partials;
            P.hist = c->hist;
            P.box = c->box;
            P.E = (int)c->E;
            P.ngroups = G.ngroups[q];
            P.nblk = G.nblk[q];
            P.active = act[m] ? 1 : 0;
            if (act[m] && (!P.r || !P.p || !P.w || !P.g || !P.x)) return NEK_E_ARG;
            G.active |= act[m] != 0;
        }
        HIP_TRY(hipMemcpyAsync(G.dtab, G.htab, G.members.size() * sizeof(BatchProb), hipMemcpyHostToDevice,
                               b->stream));
        if (G.active &&
            (rc = np_ops(G.NP)->batch_iter(b->stream, prec, v, x64, G.dtab, G.downer, G.grid, group_D(b, G, prec),
                                           0, b->dbase, false, true)))
            return rc;
        key.push_back(v);
        key.push_back((int)G.grid);
        for (char a : G.layout_act) key.push_back(a);
    }
    for (int m = 0; m < n; ++m) b->hscs[m] = act[m] ? b->ctx[m]->sc : nullptr;
    HIP_TRY(hipMemcpyAsync(b->dscs, b->hscs, n * sizeof(Scal *), hipMemcpyHostToDevice, b->stream));
    if ((rc = fill_i32(b->stream, b->dbase, -CHUNK_ITERS, 1))) return rc;
    if (use_graph && key != b->graph_key) {
        if ((rc = capture_chunk(b, prec))) return rc;
        b->graph_key = key;
    }
    if (t) HIP_TRY(hipEventRecord(b->t0, b->stream));
    int launched = 0, pend = -1, slot = 0;
    while (launched < maxcap) {
        if (use_graph)
            HIP_TRY(hipGraphLaunch(b->exec, b->stream));
        else if ((rc = enqueue_chunk(b, prec)))
            return rc;
        launched += CHUNK_ITERS;
        ++b->chunks;
        HIP_TRY(hipEventRecord(b->ev[slot], b->stream));
        if (pend >= 0) {
            // every chunk ends with k_batch_alldone writing hflags[0]
            HIP_TRY(hipEventSynchronize(b->ev[pend]));
            if (__atomic_load_n(&b->hflags[0], __ATOMIC_ACQUIRE)) break;
        }
        pend = slot;
        slot ^= 1;
    }
    for (auto &G : b->groups)
        if (G.active &&
            (rc = np_ops(G.NP)->batch_iter(b->stream, prec, G.variant[prec], x64, G.dtab, G.downer, G.grid,
                                           group_D(b, G, prec), CHUNK_ITERS + 1, b->dbase, true, false)))
            return rc;
    if (t) HIP_TRY(hipEventRecord(b->t1, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    if (t) HIP_TRY(hipEventElapsedTime(t, b->t0, b->t1));
    return NEK_OK;
}

// Scalars of the flagged members, one synchronisation.
int read_scals(nek_batch *b, const std::vector<char> &which)
{
    for (int m = 0; m < nprob(b); ++m)
        if (which[m])
            HIP_TRY(hipMemcpyAsync(&b->hscal[m], b->ctx[m]->sc, sizeof(Scal), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return NEK_OK;
}

int batch_fp64(nek_batch *b, const double *const *f, const double *const *x0, double tol, int maxit,
               double *const *x, std::vector<nek_stats> &st, bool graph)
{
    const int n = nprob(b);
    int rc;
    std::vector<char> all(n, 1);
    std::vector<void *> xs(x, x + n);
    for (int m = 0; m < n; ++m) {
        nek_ctx *c = b->ctx[m];
        if ((rc = ensure_fp64_work(c)) || (rc = ensure_hist(c, (long)maxit + 1)) ||
            (rc = cg_prologue(c, f[m], x0 ? x0[m] : nullptr, x[m], c->r64)) ||
            (rc = start_launch(c, 1, 0, tol, maxit, 0)))
            return rc;
    }
    if ((rc = run_batch(b, NEK_PREC_FP64, all, xs, maxit, graph))) return rc;
    if ((rc = read_scals(b, all))) return rc;
    std::vector<double> bb(n);
    for (int m = 0; m < n; ++m) {
        const Scal &h = b->hscal[m];
        st[m].iters = h.fin.iter;
        st[m].last_rec_res = h.hist_den > 0 ? std::sqrt(h.fin.rtz / h.hist_den) : 0.0;
        st[m].status = finish_status(h.fin, tol);
        bb[m] = h.hist_den;
    }
    // true residuals of the returned iterates, read back together
    for (int m = 0; m < n; ++m) {
        nek_ctx *c = b->ctx[m];
        if ((rc = ax_local_launch(c, x[m], c->w64, NEK_F64, NEK_PREC_FP64)) ||
            (rc = resid_launch(c, c->b, c->w64, c->r64, 1)))
            return rc;
    }
    if ((rc = read_scals(b, all))) return rc;
    for (int m = 0; m < n; ++m)
        st[m].true_rel_res = bb[m] > 0 ? std::sqrt(b->hscal[m].red[1]) / std::sqrt(bb[m]) : 0.0;
    return NEK_OK;
}

int batch_mixed(nek_batch *b, const double *const *f, const double *const *x0, double tol, int maxit,
                double *const *x, std::vector<nek_stats> &st, bool graph)
{
    const int n = nprob(b);
    const int prec = b->ctx[0]->prec;
    int rc;
    std::vector<IrCtl> S(n);
    std::vector<char> all(n, 1), act(n, 0), live(n, 0);
    std::vector<void *> xs(n, nullptr);
    for (int m = 0; m < n; ++m) {
        nek_ctx *c = b->ctx[m];
        if ((rc = ensure_mixed_work(c)) || (rc = ensure_hist(c, (long)maxit + 1))) return rc;
        ir_init(c, S[m]);
        if ((rc = cg_prologue(c, f[m], x0 ? x0[m] : nullptr, x[m], c->r64))) return rc;
        xs[m] = inner_x(c);
    }
    if ((rc = read_scals(b, all))) return rc;
    for (int m = 0; m < n; ++m) ir_start(S[m], b->hscal[m]);
    while (true) {
        int maxcap = 0;
        bool any = false;
        for (int m = 0; m < n; ++m) {
            act[m] = 0;
            if (S[m].finished) continue;
            nek_ctx *c = b->ctx[m];
            const IrStep step = ir_decide(S[m], c, tol, maxit);
            if (step == IR_DONE) {
                S[m].finished = true;
            } else if (step == IR_FALLBACK) {
                if ((rc = ir_fallback(c, S[m], tol, maxit, x[m]))) return rc;
            } else {
                int cap = 0;
                if ((rc = ir_inner_launch(c, S[m], tol, maxit, &cap))) return rc;
                act[m] = 1;
                any = true;
                maxcap = std::max(maxcap, cap);
            }
        }
        if (!any) break;
        if ((rc = run_batch(b, prec, act, xs, maxcap, graph))) return rc;
        if ((rc = read_scals(b, act))) return rc;
        for (int m = 0; m < n; ++m) {
            live[m] = 0;
            if (!act[m]) continue;
            if ((rc = ir_inner_done(b->ctx[m], S[m], b->hscal[m], x[m]))) return rc;
            live[m] = !S[m].finished;
        }
        if ((rc = read_scals(b, live))) return rc;
        for (int m = 0; m < n; ++m)
            if (live[m]) ir_outer_done(S[m], b->hscal[m]);
    }
    for (int m = 0; m < n; ++m) {
        ir_stats(S[m], &st[m]);
        st[m].status = S[m].status;
    }
    return NEK_OK;
}

}  // namespace
}  // namespace nek

extern "C" {

void nek_batch_free(nek_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    // sharers before the owners of their set-up data
    for (size_t m = b->ctx.size(); m-- > 0;) nek_free(b->ctx[m]);
    for (auto &G : b->groups) {
        dfree(G.dtab);
        dfree(G.downer);
        if (G.htab) (void)hipHostFree(G.htab);
        if (G.s) (void)hipStreamDestroy(G.s);
        if (G.join) (void)hipEventDestroy(G.join);
    }
    dfree(b->dscs);
    dfree(b->dbase);
    if (b->hscs) (void)hipHostFree(b->hscs);
    if (b->hscal) (void)hipHostFree(b->hscal);
    if (b->hflags) (void)hipHostFree(b->hflags);
    for (hipEvent_t e : {b->ev[0], b->ev[1], b->fork, b->entry, b->t0, b->t1})
        if (e) (void)hipEventDestroy(e);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

int nek_setup_batch(int n, const nek_mesh *meshes, const int *N, const nek_opts *opts, void *stream,
                    nek_batch **out)
{
    if (n < 1 || n > 4096 || !meshes || !N || !out) return NEK_E_ARG;
    if (opts && opts->precond != NEK_PC_NONE) return NEK_E_ARG;   // batches run unpreconditioned
    *out = nullptr;
    nek_batch *b = new (std::nothrow) nek_batch;
    if (!b) return NEK_E_OOM;
    b->user = (hipStream_t)stream;
    auto fail = [&](int code) { nek_batch_free(b); return code; };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return fail(NEK_E_HIP);
    // the members' setup uploads follow the caller's earlier work on its stream
    if (hipEventCreateWithFlags(&b->entry, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(b->entry, (hipStream_t)stream) != hipSuccess ||
        hipStreamWaitEvent(b->stream, b->entry, 0) != hipSuccess)
        return fail(NEK_E_HIP);
    b->ctx.assign(n, nullptr);
    b->root.assign(n, 0);
    b->epw_opt = opts ? opts->elts_per_wg : 0;
    for (int m = 0; m < n; ++m) {
        int k = 0;
        while (k < m && !(b->root[k] == k && N[k] == N[m] && same_mesh(meshes[k], meshes[m]))) ++k;
        b->root[m] = k;
        const int rc = k < m ? setup_shared(b->ctx[k], opts, b->stream, &b->ctx[m])
                             : nek_setup(&meshes[m], N[m], opts, b->stream, &b->ctx[m]);
        if (rc) return fail(rc);
        // members follow the batch's configuration and never tune alone
        b->ctx[m]->batch_member = true;
        for (int q = 0; q < 3; ++q) b->ctx[m]->tuned[q] = true;
    }
    // The K problems on one mesh share the persistent grid of one solo
    // launch: each gets 1/K of it (never less than its element groups allow),
    // so their K blocks per XCD slot run in one round, with the factors of an
    // element group read from HBM once and from L2 by the others.  Each
    // member context keeps that grid for its own solves too, which therefore
    // reproduce its batched result bit for bit.
    for (int m = 0; m < n; ++m) {
        int K = 0;
        for (int k = 0; k < n; ++k) K += b->root[k] == b->root[m];
        if (K > 1) b->ctx[m]->ax_wg = (int)((8L * num_cu() + K - 1) / K);
    }
    b->group_of.assign(n, -1);
    for (int NP = 2; NP <= MAX_NP; ++NP) {
        Group G;
        G.NP = NP;
        for (int m = 0; m < n; ++m)
            if (N[m] + 1 == NP) G.members.push_back(m);
        if (G.members.empty()) continue;
        for (int m : G.members) b->group_of[m] = (int)b->groups.size();
        b->groups.push_back(std::move(G));
    }
    for (auto &G : b->groups) {
        if (b->epw_opt != 0) {
            const int v = b->ctx[G.members[0]]->variant[0];   // set by nek_setup from elts_per_wg
            for (int q = 0; q < 3; ++q) G.variant[q] = v;
            b->tuned[0] = b->tuned[1] = b->tuned[2] = true;
        }
        if (dalloc(G.dtab, G.members.size())) return fail(NEK_E_OOM);
        if (hipHostMalloc((void **)&G.htab, G.members.size() * sizeof(BatchProb), hipHostMallocDefault) != hipSuccess)
            return fail(NEK_E_OOM);
        if (hipStreamCreateWithFlags(&G.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&G.join, hipEventDisableTiming) != hipSuccess)
            return fail(NEK_E_HIP);
    }
    if (dalloc(b->dscs, n) || dalloc(b->dbase, 1)) return fail(NEK_E_OOM);
    if (hipHostMalloc((void **)&b->hscs, n * sizeof(Scal *), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->hscal, n * sizeof(Scal), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->hflags, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(NEK_E_OOM);
    b->hflags[0] = b->hflags[1] = 0;
    if (hipHostGetDevicePointer((void **)&b->dflag, b->hflags, 0) != hipSuccess) return fail(NEK_E_HIP);
    for (hipEvent_t *e : {&b->ev[0], &b->ev[1], &b->fork})
        if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) return fail(NEK_E_HIP);
    if (hipEventCreate(&b->t0) != hipSuccess || hipEventCreate(&b->t1) != hipSuccess) return fail(NEK_E_HIP);
    if (hipStreamSynchronize(b->stream) != hipSuccess) return fail(NEK_E_HIP);
    *out = b;
    return NEK_OK;
}

int nek_batch_size(const nek_batch *b) { return b ? (int)b->ctx.size() : NEK_E_ARG; }

int nek_batch_ctx(nek_batch *b, int i, nek_ctx **out)
{
    if (!b || !out || i < 0 || i >= nprob(b)) return NEK_E_ARG;
    *out = b->ctx[i];
    return NEK_OK;
}

int nek_batch_mesh_of(const nek_batch *b, int i)
{
    if (!b || i < 0 || i >= nprob(b)) return NEK_E_ARG;
    return b->root[i];
}

int nek_batch_set_variant(nek_batch *b, int prec, int N, int variant)
{
    if (!b || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G) return NEK_E_ARG;
    for (auto &G : b->groups) {
        if (G.NP != N + 1) continue;
        if (variant < 0 || variant >= np_ops(G.NP)->nvariants) return NEK_E_ARG;
        G.variant[prec] = variant;
        for (int m : G.members) b->ctx[m]->variant[prec] = variant;
        b->tuned[prec] = true;   // an explicit choice: no autotuning at the next solve
        return NEK_OK;
    }
    return NEK_E_ARG;
}

int nek_batch_get_variant(const nek_batch *b, int prec, int i, int *variant)
{
    if (!b || !variant || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G || i < 0 || i >= nprob(b))
        return NEK_E_ARG;
    *variant = b->groups[b->group_of[i]].variant[prec];
    return NEK_OK;
}

int nek_batch_orders(const nek_batch *b, int *N_out)
{
    if (!b) return NEK_E_ARG;
    if (N_out)
        for (size_t g = 0; g < b->groups.size(); ++g) N_out[g] = b->groups[g].NP - 1;
    return (int)b->groups.size();
}

int nek_batch_tune(nek_batch *b, int prec, int iters, double *us_per_iter)
{
    if (!b || prec < NEK_PREC_FP64 || prec > NEK_PREC_BF16G || iters < 2) return NEK_E_ARG;
    const int n = nprob(b);
    int rc;
    std::vector<void *> xs(n, nullptr);
    for (int m = 0; m < n; ++m) {
        nek_ctx *c = b->ctx[m];
        if ((rc = ensure_fp64_work(c)) || (rc = ensure_g(c, prec)) || (rc = ensure_hist(c, iters + 1))) return rc;
        if (prec == NEK_PREC_FP64 ? dalloc(c->d64, c->nl)
                                  : ((c->opts.corr_fp32 ? dalloc(c->d32, c->nl) : dalloc(c->d64, c->nl)) ||
                                     dalloc(c->r32, c->nl) || dalloc(c->p32, c->nl) || dalloc(c->w32, c->nl)))
            return NEK_E_OOM;
        // synthetic SPD system: b = M dssum(1), x0 = 0
        if ((rc = fill_f64(c, c->w64, 1.0, c->nl)) || (rc = gather_launch(c, c->w64, c->b, false)) ||
            (rc = glsc3_to_slot(c, c->b, c->b, NEK_F64, 0)))
            return rc;
        xs[m] = prec == NEK_PREC_FP64 ? (void *)c->d64 : inner_x(c);
    }
    if (us_per_iter)
        for (size_t k = 0; k < NEK_MAX_VARIANTS * b->groups.size(); ++k) us_per_iter[k] = 0.0;
    int slot = 0;
    for (auto &G : b->groups) {
        std::vector<char> act(n, 0);
        for (int m : G.members) act[m] = 1;
        const int nv = np_ops(G.NP)->nvariants;
        double best_t = INFINITY;
        int best_v = G.variant[prec];
        for (int v = 0; v < nv; ++v) {
            G.variant[prec] = v;
            float ms = 0;
            for (int rep = 0; rep < 2; ++rep) {   // the first pass warms up
                for (int m : G.members) {
                    nek_ctx *c = b->ctx[m];
                    if (prec == NEK_PREC_FP64) {
                        HIP_TRY(hipMemcpyAsync(c->r64, c->b, c->nl * sizeof(double), hipMemcpyDeviceToDevice,
                                               b->stream));
                        if ((rc = glsc3_to_slot(c, c->r64, c->r64, NEK_F64, 1)) ||
                            (rc = fill_f64(c, c->d64, 0.0, c->nl)))
                            return rc;
                    } else {
                        if ((rc = ops(c)->inner_start(c, c->b, c->r32, inner_x(c), !c->opts.corr_fp32)) ||
                            (rc = red_final(c, 1)))
                            return rc;
                    }
                    if ((rc = start_launch(c, 1, 0, 0.0, iters, 0))) return rc;
                }
                if ((rc = run_batch(b, prec, act, xs, iters, false, &ms))) return rc;
            }
            const double t = 1e3 * ms / iters;
            if (us_per_iter) us_per_iter[slot + v] = t;
            if (t < best_t) {
                best_t = t;
                best_v = v;
            }
        }
        G.variant[prec] = best_v;
        for (int m : G.members) b->ctx[m]->variant[prec] = best_v;
        slot += NEK_MAX_VARIANTS;
    }
    b->tuned[prec] = true;
    drop_graph(b);
    return NEK_OK;
}

int nek_cg_solve_batch(nek_batch *b, const double *const *f, const double *const *x0, double tol, int maxit,
                       double *const *x, nek_stats *stats, int flags)
{
    if (!b || !f || !x || maxit < 0) return NEK_E_ARG;
    const int n = nprob(b);
    const int prec = b->ctx[0]->prec;
    for (int m = 0; m < n; ++m)
        if (!f[m] || !x[m] || b->ctx[m]->prec != prec || b->ctx[m]->precond || b->ctx[m]->geom) return NEK_E_ARG;
    const bool graph = !(flags & NEK_BATCH_NO_GRAPH);
    // the solve follows the caller's earlier work on its stream
    HIP_TRY(hipEventRecord(b->entry, b->user));
    HIP_TRY(hipStreamWaitEvent(b->stream, b->entry, 0));
    std::vector<nek_stats> st(n);
    const auto t0 = std::chrono::steady_clock::now();
    if (b->epw_opt == 0 && !b->tuned[prec]) {
        const int rt = nek_batch_tune(b, prec, 20, nullptr);
        if (rt) return rt;
    }
    int rc = prec == NEK_PREC_FP64 ? batch_fp64(b, f, x0, tol, maxit, x, st, graph)
                                   : batch_mixed(b, f, x0, tol, maxit, x, st, graph);
    if (hipStreamSynchronize(b->stream) != hipSuccess && rc >= 0) rc = NEK_E_HIP;
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (rc < 0) return rc;
    int worst = NEK_OK;
    for (int m = 0; m < n; ++m) {
        st[m].t_solve_s = t;
        if (st[m].status < 0 && (worst >= 0 || st[m].status < worst)) worst = st[m].status;
        else if (st[m].status == NEK_NOCONV && worst == NEK_OK) worst = NEK_NOCONV;
        if (stats) stats[m] = st[m];
    }
    return worst;
}

int nek_batch_counters(const nek_batch *b, int64_t *chunks, int64_t *captures)
{
    if (!b) return NEK_E_ARG;
    if (chunks) *chunks = b->chunks;
    if (captures) *captures = b->captures;
    return NEK_OK;
}

}  // extern "C"
