// dba_host.cpp -- C ABI, validation, device layout builder, iteration driver
// (eager launches or hipGraph replay), launch-schedule autotuner and kernel
// timing for the ADMM bundle-adjustment library.
#include "dba_host_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

namespace dba {
namespace host {

void drop_graphs(dba_handle *h)
{
    for (auto &g : h->gexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    for (auto &row : h->tgraph)
        for (TimedGraph &t : row) {
            if (t.exec) (void)hipGraphExecDestroy(t.exec);
            for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
            t = TimedGraph();
        }
    h->tgraph_next[0] = h->tgraph_next[1] = 0;
    for (auto &g : h->sgexec) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

int validate(dba_handle *h, int p, const dba_problem_desc &d)
{
    std::string msg;
    const int rc = dba::validate_problem(p, d, h->opt.camera_model, &msg);
    if (rc != DBA_OK) return fail(h, rc, "%s", msg.c_str());
    return DBA_OK;
}

template <typename R>
int build_set(dba_handle *h, int np, const dba_problem_desc *probs, ProblemSet *ps, DevArrays<R> &A)
{
    using R2 = typename dba::Vec<R>::R2;
    static_assert(sizeof(R2) == 2 * sizeof(R) && sizeof(dba::PtCopy<R>) == 3 * sizeof(R) &&
                      sizeof(double4) == 4 * sizeof(double),
                  "flattened host arrays match the device vector types");
    dba::LayoutOptions lo;
    lo.camera_blocks = h->opt.camera_blocks;
    lo.block_points = h->opt.block_points;
    lo.block_cameras = h->opt.block_cameras;
    lo.camera_model = h->opt.camera_model;
    dba::Layout<R> lay;
    std::string msg;
    const int lrc = dba::build_layout<R>(lo, np, probs, &lay, &msg);
    if (lrc != DBA_OK) return fail(h, lrc, "%s", msg.c_str());
    const bool per_obs = !h->opt.camera_blocks;
    const bool k2 = lay.n_blocks2 > 0;
    ps->n_problems = np;
    ps->ranges = lay.ranges;
    for (int p = 0; p < np; ++p) {
        ps->m.push_back(probs[p].n_cams);
        ps->n.push_back(probs[p].n_points);
        ps->L.push_back(probs[p].n_obs);
    }
    const long long S = lay.n_slots, n_chunks = lay.n_chunks, n_recs = lay.n_recs;
    const int n_cams = lay.n_cams, n_pts = lay.n_pts, n_cw = lay.n_cw;
    ps->n_slots = S;
    const size_t SY = per_obs ? (size_t)S : 0;
    std::vector<uint8_t> mask(S, 1);
    std::vector<Ctrl> ctrl(np);
    for (int p = 0; p < np; ++p) {
        Ctrl &c = ctrl[p];
        std::memset(&c, 0, sizeof(c));
        c.rho_x = h->opt.rho_x;
        c.rho_y = h->opt.rho_y;
        c.ratio_x = c.ratio_y = 1.0;
        c.last_rho_x = h->opt.rho_x;
        c.last_rho_y = h->opt.rho_y;
        c.rb_mu = h->opt.rb_mu;
        c.rb_tau = h->opt.rb_tau;
        c.rho_min = h->opt.rho_min;
        c.rho_max = h->opt.rho_max;
        c.balancing = h->opt.rho_balancing ? 1 : 0;
    }
    const std::vector<int> &pt_off = lay.pt_off, &chunk_cam = lay.chunk_cam, &chunk_prob = lay.chunk_prob,
                           &cam_prob = lay.cam_prob,
                           &pt_prob = lay.pt_prob, &cam_chunk0 = lay.cam_chunk0, &cam_count = lay.cam_count,
                           &cw_pt0 = lay.cw_pt0, &pslot = lay.pslot,
                           &ptid = lay.ptid, &orig = lay.orig, &blk_chunk = lay.blk_chunk, &blk_rec = lay.blk_rec,
                           &blk_cam = lay.blk_cam, &blk_prob = lay.blk_prob, &blk_pt = lay.blk_pt;
    const std::vector<double> &cons_y = lay.cons_y;
    const std::vector<R> &copy_y = lay.copy_y, &copy_yc = lay.copy_yc;

    // device
    Buffers &B = ps->buf;
    R2 *d_uv; int *d_pslot, *d_ptid, *d_orig; uint8_t *d_mask; R *d_copy; double *d_dual;
    dba::PtCopy<R> *d_xrec; dba::PtDual *d_urec; int *d_ptoff, *d_chunk_cam, *d_chunk_prob, *d_cam_prob, *d_pt_prob, *d_cam_chunk0, *d_cam_count;
    double *d_cons_y; double4 *d_cons_x; Ctrl *d_ctrl; ProblemRange *d_prob;
    double *d_cpart, *d_ppart, *d_campart, *d_epart, *d_estats;
    int *d_cw_pt0;
    HIP_TRY(h, B.alloc(&d_uv, S));
    HIP_TRY(h, B.alloc(&d_pslot, S));
    HIP_TRY(h, B.alloc(&d_ptid, S));
    HIP_TRY(h, B.alloc(&d_orig, S));
    HIP_TRY(h, B.alloc(&d_mask, S));
    HIP_TRY(h, B.alloc(&d_copy, 9 * SY));
    HIP_TRY(h, B.alloc(&d_dual, 9 * SY));
    HIP_TRY(h, B.alloc(&d_xrec, n_recs));
    HIP_TRY(h, B.alloc(&d_urec, n_recs));
    HIP_TRY(h, B.alloc(&d_ptoff, n_pts + 1));
    HIP_TRY(h, B.alloc(&d_chunk_cam, n_chunks));
    HIP_TRY(h, B.alloc(&d_chunk_prob, n_chunks));
    HIP_TRY(h, B.alloc(&d_cam_prob, n_cams));
    HIP_TRY(h, B.alloc(&d_pt_prob, n_pts));
    HIP_TRY(h, B.alloc(&d_cam_chunk0, n_cams + 1));
    HIP_TRY(h, B.alloc(&d_cam_count, n_cams));
    HIP_TRY(h, B.alloc(&d_cons_y, (size_t)n_cams * dba::kConsY));
    HIP_TRY(h, B.alloc(&d_cons_x, n_pts));
    HIP_TRY(h, B.alloc(&d_ctrl, np));
    HIP_TRY(h, B.alloc(&d_prob, np));
    HIP_TRY(h, B.alloc(&d_cpart, (size_t)n_chunks * dba::kCpart));
    HIP_TRY(h, B.alloc(&d_ppart, 2 * (size_t)(n_cw / dba::kConsWaves)));
    HIP_TRY(h, B.alloc(&d_cw_pt0, n_cw + 1));
    HIP_TRY(h, hipMemcpy(d_cw_pt0, cw_pt0.data(), (n_cw + 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, B.alloc(&d_campart, 2 * (size_t)n_cams));
    HIP_TRY(h, B.alloc(&d_epart, (size_t)n_chunks * dba::kEpart));
    HIP_TRY(h, B.alloc(&d_estats, (size_t)np * dba::kEpart));

    HIP_TRY(h, hipMemcpy(d_uv, lay.uv.data(), S * sizeof(R2), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_pslot, pslot.data(), S * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_ptid, ptid.data(), S * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_orig, orig.data(), S * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_mask, mask.data(), S, hipMemcpyHostToDevice));
    if (per_obs) {
        HIP_TRY(h, hipMemcpy(d_copy, copy_y.data(), 9 * SY * sizeof(R), hipMemcpyHostToDevice));
        HIP_TRY(h, hipMemset(d_dual, 0, 9 * SY * sizeof(double)));
    }
    HIP_TRY(h, hipMemcpy(d_xrec, lay.xrec.data(), n_recs * sizeof(dba::PtCopy<R>), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(d_urec, 0, n_recs * sizeof(dba::PtDual)));
    HIP_TRY(h, hipMemcpy(d_ptoff, pt_off.data(), (n_pts + 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_chunk_cam, chunk_cam.data(), n_chunks * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_chunk_prob, chunk_prob.data(), n_chunks * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_cam_prob, cam_prob.data(), n_cams * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_pt_prob, pt_prob.data(), n_pts * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_cam_chunk0, cam_chunk0.data(), (n_cams + 1) * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_cam_count, cam_count.data(), n_cams * sizeof(int), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_cons_y, cons_y.data(), cons_y.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_cons_x, lay.cons_x.data(), n_pts * sizeof(double4), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_ctrl, ctrl.data(), np * sizeof(Ctrl), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(d_prob, ps->ranges.data(), np * sizeof(ProblemRange), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(d_cpart, 0, (size_t)n_chunks * dba::kCpart * sizeof(double)));
    R *d_copy_yc;
    double *d_dual_yc;
    HIP_TRY(h, B.alloc(&d_copy_yc, 9 * (size_t)n_chunks));
    HIP_TRY(h, B.alloc(&d_dual_yc, 9 * (size_t)n_chunks));
    HIP_TRY(h, hipMemcpy(d_copy_yc, copy_yc.data(), 9 * (size_t)n_chunks * sizeof(R), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemset(d_dual_yc, 0, 9 * (size_t)n_chunks * sizeof(double)));
    int *d_blk_chunk = nullptr, *d_blk_rec = nullptr, *d_blk_cam = nullptr, *d_blk_prob = nullptr,
        *d_blk_pt = nullptr;
    if (k2) {
        auto up = [&](int **d, const std::vector<int> &v) -> hipError_t {
            hipError_t e = B.alloc(d, v.size());
            if (e == hipSuccess) e = hipMemcpy(*d, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
            return e;
        };
        HIP_TRY(h, up(&d_blk_chunk, blk_chunk));
        HIP_TRY(h, up(&d_blk_rec, blk_rec));
        HIP_TRY(h, up(&d_blk_cam, blk_cam));
        HIP_TRY(h, up(&d_blk_prob, blk_prob));
        HIP_TRY(h, up(&d_blk_pt, blk_pt));
    }
    A.n_blocks2 = lay.n_blocks2;
    A.blk_chunk = d_blk_chunk;
    A.blk_rec = d_blk_rec;
    A.blk_cam = d_blk_cam;
    A.blk_prob = d_blk_prob;
    A.blk_pt = d_blk_pt;
    A.camera_blocks = h->opt.camera_blocks ? 1 : 0;
    A.copy_yc = d_copy_yc;
    A.dual_yc = d_dual_yc;

    A.n_slots = S;
    A.uv = d_uv; A.pslot = d_pslot; A.ptid = d_ptid;
    A.copy_y = d_copy; A.dual_y = d_dual; A.mask = d_mask; A.slot_orig = d_orig;
    A.n_recs = n_recs; A.xrec = d_xrec; A.urec = d_urec; A.pt_off = d_ptoff;
    A.n_chunks = (int)n_chunks; A.n_cams = n_cams; A.n_pts = n_pts; A.n_problems = np;
    A.chunk_cam = d_chunk_cam; A.chunk_prob = d_chunk_prob; A.cam_prob = d_cam_prob; A.pt_prob = d_pt_prob;
    A.cam_chunk0 = d_cam_chunk0; A.cam_count = d_cam_count;
    A.cons_y = d_cons_y; A.cons_x = d_cons_x; A.ctrl = d_ctrl; A.prob = d_prob;
    A.n_cw = n_cw; A.cw_pt0 = d_cw_pt0;
    A.cpart = d_cpart; A.ppart = d_ppart; A.campart = d_campart; A.epart = d_epart; A.estats = d_estats;
    ps->mask = d_mask;
    return DBA_OK;
}

void free_mlp(dba_handle *h);

// The local-solve launch of the handle's start mode.
template <typename R>
hipError_t launch_local_sel(dba_handle *h, const DevArrays<R> &A, int bw, int pers)
{
    if constexpr (std::is_same<R, float>::value) {
        if (h->start == DBA_START_LEARNED)
            return dba::launch_local_learned(A, h->sp, h->mlp->params(), pers, h->n_cu, h->stream);
    }
    if (h->opt.camera_blocks) return dba::launch_local_block<R>(A, h->sp, bw, pers, h->n_cu, h->stream);
    return dba::launch_local<R>(A, h->sp, bw, pers, h->n_cu, h->stream);
}

// One ADMM iteration: the three launches on the handle's stream.  mark(kid)
// is called before each launch with its kernel id and returns the event to
// record after it (recording its start event itself), or nullptr; external
// records those events as event-record nodes of a graph being captured.
template <typename R, typename Mark>
hipError_t run_iteration_marked(dba_handle *h, const DevArrays<R> &A, int bw, int pers, Mark mark,
                                bool external = false)
{
    auto done = [&](hipEvent_t e1) {
        if (!e1) return;
        if (external)
            (void)hipEventRecordWithFlags(e1, h->stream, hipEventRecordExternal);
        else
            (void)hipEventRecord(e1, h->stream);
    };
    hipEvent_t e;
    hipError_t err;
    e = mark(h->start == DBA_START_LEARNED ? 3 : 0);
    err = launch_local_sel<R>(h, A, bw, pers);
    done(e);
    if (err != hipSuccess) return err;
    e = mark(1);
    err = dba::launch_consensus<R>(A, h->seg_sched, h->stream);
    done(e);
    if (err != hipSuccess) return err;
    e = mark(2);
    err = dba::launch_norms<R>(A, h->stream);
    done(e);
    return err;
}

inline hipEvent_t no_mark(int) { return nullptr; }

// Eager iteration; with timed, each kernel between two events of the
// handle's pool (read by collect_timing).
// The next two events of the handle's pool for kernel kid (read by
// collect_timing); false if the pool cannot grow.
bool pool_pair(dba_handle *h, int kid, hipEvent_t *e0, hipEvent_t *e1)
{
    Timing &T = h->timing;
    if (T.used + 2 > T.pool.size()) {
        for (int q = 0; q < 64; ++q) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return false;
            T.pool.push_back(e);
        }
    }
    *e0 = T.pool[T.used];
    *e1 = T.pool[T.used + 1];
    T.pending_kernel.push_back(kid);
    T.used += 2;
    return true;
}

template <typename R>
hipError_t run_iteration(dba_handle *h, const DevArrays<R> &A, int bw, int pers, bool timed)
{
    if (!timed) return run_iteration_marked<R>(h, A, bw, pers, no_mark);
    auto mark = [&](int kid) -> hipEvent_t {
        if (!(h->timing.mask >> kid & 1u)) return nullptr;
        hipEvent_t e0, e1;
        if (!pool_pair(h, kid, &e0, &e1)) return nullptr;
        (void)hipEventRecord(e0, h->stream);
        return e1;
    };
    return run_iteration_marked<R>(h, A, bw, pers, mark);
}

int collect_timing(dba_handle *h);

// Reads a launched timed graph's kernel times (waits for its last event).
int collect_graph_times(dba_handle *h, TimedGraph &g)
{
    if (!g.pending) return DBA_OK;
    HIP_TRY(h, hipEventSynchronize(g.ev.back()));
    for (size_t q = 0; q < g.kid.size(); ++q) {
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, g.ev[2 * q], g.ev[2 * q + 1]));
        h->timing.total_ms[g.kid[q]] += ms;
        h->timing.launches[g.kid[q]] += 1;
    }
    g.pending = false;
    return DBA_OK;
}

// Captures the four timed graphs (1 and kGraphBatch iterations, two of
// each).  false (and timed graphs off for the handle) if the capture of
// event records is refused.
template <typename R>
bool timed_graphs_ready(dba_handle *h, const DevArrays<R> &A)
{
    if (h->tgraph[0][0].exec && h->tgraph_mask != h->timing.mask) {
        if (collect_timing(h) != DBA_OK) return false;
        drop_graphs(h);
    }
    h->tgraph_mask = h->timing.mask;
    for (int sz = 0; sz < 2; ++sz)
        for (int b = 0; b < 2; ++b) {
            TimedGraph &g = h->tgraph[sz][b];
            if (g.exec) continue;
            const int iters = sz == 0 ? 1 : kGraphBatch;
            bool ok = true;
            int cur = 0;  // iteration of the graph being captured
            auto mark = [&](int kid) -> hipEvent_t {
                if (!(h->timing.mask >> kid & 1u)) return nullptr;
                if ((h->timing.mask & kFirstOnly) && cur > 0) return nullptr;
                hipEvent_t e0, e1;
                if (hipEventCreate(&e0) != hipSuccess) { ok = false; return nullptr; }
                if (hipEventCreate(&e1) != hipSuccess) {
                    (void)hipEventDestroy(e0);
                    ok = false;
                    return nullptr;
                }
                g.ev.push_back(e0);
                g.ev.push_back(e1);
                g.kid.push_back(kid);
                if (hipEventRecordWithFlags(e0, h->stream, hipEventRecordExternal) != hipSuccess) ok = false;
                return e1;
            };
            hipGraph_t graph = nullptr;
            if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) ok = false;
            hipError_t err = hipSuccess;
            for (int it = 0; ok && it < iters && err == hipSuccess; ++it) {
                cur = it;
                err = run_iteration_marked<R>(h, A, h->block_waves, h->persistent, mark, true);
            }
            hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
            ok = ok && err == hipSuccess && e2 == hipSuccess && graph;
            if (ok) ok = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) == hipSuccess;
            if (graph) (void)hipGraphDestroy(graph);
            if (!ok) {
                (void)hipGetLastError();
                drop_graphs(h);
                h->tgraph_off = true;
                return false;
            }
        }
    return true;
}

// Timed iterations replayed from the timed graphs; every replay's times are
// read before its graph is launched again and at the end.
template <typename R>
int iterate_timed_graphs(dba_handle *h, int n)
{
    auto launch = [&](int sz) -> int {
        TimedGraph &g = h->tgraph[sz][h->tgraph_next[sz]];
        int rc = collect_graph_times(h, g);
        if (rc != DBA_OK) return rc;
        HIP_TRY(h, hipGraphLaunch(g.exec, h->stream));
        g.pending = true;
        h->tgraph_next[sz] ^= 1;
        return DBA_OK;
    };
    int rc = DBA_OK;
    for (; rc == DBA_OK && n >= kGraphBatch; n -= kGraphBatch) rc = launch(1);
    for (; rc == DBA_OK && n > 0; --n) rc = launch(0);
    if (rc != DBA_OK) return rc;
    return collect_timing(h);
}

// Sampled timing without event-record nodes inside graphs (which some HIP
// runtimes refuse to capture): the local launch of the first iteration of a
// batch is launched directly between two events recorded on the stream, and
// the rest of the iteration -- or of a batch of kGraphBatch iterations -- is
// replayed from a graph.  false if a capture fails.
template <typename R>
bool sampled_graphs_ready(dba_handle *h, const DevArrays<R> &A)
{
    if (h->sgexec[0]) return true;
    for (int g = 0; g < 2; ++g) {
        hipGraph_t graph = nullptr;
        hipError_t err = hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) {
            err = dba::launch_consensus<R>(A, h->seg_sched, h->stream);
            if (err == hipSuccess) err = dba::launch_norms<R>(A, h->stream);
            for (int it = 1; g == 1 && it < kGraphBatch && err == hipSuccess; ++it)
                err = run_iteration<R>(h, A, h->block_waves, h->persistent, false);
            const hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
            if (err == hipSuccess) err = e2;
        }
        if (err == hipSuccess && graph) err = hipGraphInstantiate(&h->sgexec[g], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (err != hipSuccess || !h->sgexec[g]) {
            (void)hipGetLastError();
            for (auto &x : h->sgexec) {
                if (x) (void)hipGraphExecDestroy(x);
                x = nullptr;
            }
            return false;
        }
    }
    return true;
}

// n sampled-timing iterations: batches of kGraphBatch, then single
// iterations; each batch's first local launch between two events, the rest
// of the batch from a graph.
template <typename R>
int iterate_sampled(dba_handle *h, const DevArrays<R> &A, int n)
{
    const int kid = h->start == DBA_START_LEARNED ? 3 : 0;
    while (n > 0) {
        const int batch = n >= kGraphBatch ? kGraphBatch : 1;
        hipEvent_t e0, e1;
        if (!pool_pair(h, kid, &e0, &e1)) return fail(h, DBA_E_DEVICE, "timing events: out of events");
        HIP_TRY(h, hipEventRecord(e0, h->stream));
        HIP_TRY(h, launch_local_sel<R>(h, A, h->block_waves, h->persistent));
        HIP_TRY(h, hipEventRecord(e1, h->stream));
        HIP_TRY(h, hipGraphLaunch(h->sgexec[batch == 1 ? 0 : 1], h->stream));
        n -= batch;
    }
    return collect_timing(h);
}

int collect_timing(dba_handle *h)
{
    Timing &T = h->timing;
    for (auto &row : h->tgraph)
        for (TimedGraph &g : row) {
            int rc = collect_graph_times(h, g);
            if (rc != DBA_OK) return rc;
        }
    if (T.used == 0) return DBA_OK;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    for (size_t q = 0; q < T.pending_kernel.size(); ++q) {
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, T.pool[2 * q], T.pool[2 * q + 1]));
        T.total_ms[T.pending_kernel[q]] += ms;
        T.launches[T.pending_kernel[q]] += 1;
    }
    T.pending_kernel.clear();
    T.used = 0;
    return DBA_OK;
}

template <typename R>
int iterate_impl(dba_handle *h, const DevArrays<R> &A, int n)
{
    static const int cand_bw[] = {1, 2, 4, 8, 1, 2, 4, 8};
    static const int cand_p[] = {0, 0, 0, 0, 1, 1, 1, 1};
    // autotune on real iterations: every schedule gives bitwise-identical
    // results, so tuning does not change the trajectory
    while (!h->schedule_ready && n > 0) {
        const bool tune_bw = h->opt.block_waves == 0, tune_p = h->opt.persistent < 0;
        std::vector<int> idx;
        for (int q = 0; q < 8; ++q)
            if ((tune_bw || cand_bw[q] == h->opt.block_waves) && (tune_p || cand_p[q] == h->opt.persistent))
                idx.push_back(q);
        if (h->tune_next == 0) {  // warm-up iteration, untimed
            HIP_TRY(h, run_iteration<R>(h, A, cand_bw[idx[0]], cand_p[idx[0]], false));
            h->tune_next = 1;
            h->tune_ms.clear();
            --n;
            continue;
        }
        const int q = idx[h->tune_next - 1];
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float ms = 0.f;
        hipError_t err = hipEventCreate(&e0);
        if (err == hipSuccess) err = hipEventCreate(&e1);
        if (err == hipSuccess) err = hipEventRecord(e0, h->stream);
        if (err == hipSuccess) err = launch_local_sel<R>(h, A, cand_bw[q], cand_p[q]);
        if (err == hipSuccess) err = hipEventRecord(e1, h->stream);
        if (err == hipSuccess) err = dba::launch_consensus<R>(A, h->seg_sched, h->stream);
        if (err == hipSuccess) err = dba::launch_norms<R>(A, h->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (err != hipSuccess) return fail(h, DBA_E_DEVICE, "schedule tuning: %s", hipGetErrorString(err));
        h->tune_ms.push_back(ms);
        --n;
        if (++h->tune_next > (int)idx.size()) {
            int best = 0;
            for (int t = 1; t < (int)h->tune_ms.size(); ++t)
                if (h->tune_ms[t] < h->tune_ms[best]) best = t;
            h->block_waves = cand_bw[idx[best]];
            h->persistent = cand_p[idx[best]];
            h->tuned = (int)idx.size();
            h->schedule_ready = true;
        }
    }
    // then the segment schedule of the consensus, on real iterations with
    // the local schedule fixed; its candidates are bitwise identical too
    static const int cand_seg[] = {1, 2, 3};
    constexpr int n_seg = (int)(sizeof(cand_seg) / sizeof(cand_seg[0]));
    while (!h->seg_ready && n > 0) {
        const int q = h->seg_next;
        h->seg_sched = cand_seg[q];
        hipEvent_t e0 = nullptr, e1 = nullptr;
        float ms = 0.f;
        hipError_t err = hipEventCreate(&e0);
        if (err == hipSuccess) err = hipEventCreate(&e1);
        if (err == hipSuccess) err = launch_local_sel<R>(h, A, h->block_waves, h->persistent);
        if (err == hipSuccess) err = hipEventRecord(e0, h->stream);
        if (err == hipSuccess) err = dba::launch_consensus<R>(A, h->seg_sched, h->stream);
        if (err == hipSuccess) err = hipEventRecord(e1, h->stream);
        if (err == hipSuccess) err = dba::launch_norms<R>(A, h->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (err != hipSuccess) return fail(h, DBA_E_DEVICE, "segment schedule tuning: %s", hipGetErrorString(err));
        h->seg_ms.push_back(ms);
        --n;
        if (++h->seg_next == n_seg) {
            int best = 0;
            for (int t = 1; t < n_seg; ++t)
                if (h->seg_ms[t] < h->seg_ms[best]) best = t;
            h->seg_sched = cand_seg[best];
            h->seg_tuned = n_seg;
            h->seg_ready = true;
        }
    }
    if (n <= 0) return DBA_OK;
    if (h->timing.on && (h->timing.mask & kFirstOnly) && h->opt.use_graph && !h->sgraph_off) {
        if (sampled_graphs_ready<R>(h, A)) return iterate_sampled<R>(h, A, n);
        h->sgraph_off = true;
    }
    if (h->timing.on && h->opt.use_graph && !h->tgraph_off && timed_graphs_ready<R>(h, A))
        return iterate_timed_graphs<R>(h, n);
    if (h->timing.on || !h->opt.use_graph) {
        for (int it = 0; it < n; ++it) HIP_TRY(h, run_iteration<R>(h, A, h->block_waves, h->persistent, h->timing.on));
        if (h->timing.on) return collect_timing(h);
        return DBA_OK;
    }
    for (int g = 0; g < 2; ++g) {
        if (h->gexec[g]) continue;
        const int iters = g == 0 ? 1 : kGraphBatch;
        hipGraph_t graph;
        HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (int it = 0; it < iters && err == hipSuccess; ++it)
            err = run_iteration<R>(h, A, h->block_waves, h->persistent, false);
        hipError_t e2 = hipStreamEndCapture(h->stream, &graph);
        if (err != hipSuccess || e2 != hipSuccess) {
            if (e2 == hipSuccess && graph) (void)hipGraphDestroy(graph);
            return fail(h, DBA_E_DEVICE, "graph capture: %s", hipGetErrorString(err != hipSuccess ? err : e2));
        }
        err = hipGraphInstantiate(&h->gexec[g], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_TRY(h, err);
    }
    while (n >= kGraphBatch) {
        HIP_TRY(h, hipGraphLaunch(h->gexec[1], h->stream));
        n -= kGraphBatch;
    }
    for (; n > 0; --n) HIP_TRY(h, hipGraphLaunch(h->gexec[0], h->stream));
    return DBA_OK;
}

void free_set(dba_handle *h)
{
    drop_graphs(h);
    delete h->ps;
    h->ps = nullptr;
}

int check_problem(const dba_handle *h, int p)
{
    if (!h->ps) return DBA_E_STATE;
    if (p < 0 || p >= h->ps->n_problems) return DBA_E_INVALID_ARG;
    return DBA_OK;
}

}  // namespace host
}  // namespace dba

using namespace dba::host;

// ============================================================================
extern "C" {

int dba_default_options(dba_options *o)
{
    if (!o) return DBA_E_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->stream = nullptr;
    o->precision = DBA_PREC_FP64;
    o->loss = DBA_LOSS_HUBER;
    o->loss_param = 2.0;
    o->rho_x = o->rho_y = 1.0;
    o->rho_balancing = 0;
    o->rb_mu = 10.0;
    o->rb_tau = 2.0;
    o->rho_min = 1e-6;
    o->rho_max = 1e6;
    o->lm_steps = 5;
    o->lm_lambda0 = 1e-3;
    o->start = DBA_START_PLAIN;
    o->learned_lm_steps = 2;
    o->use_graph = 1;
    o->block_waves = 0;
    o->persistent = -1;
    o->camera_blocks = 0;
    o->block_points = 0;
    o->camera_model = DBA_CAMERA_ANGLE_AXIS;
    o->local_solver = DBA_SOLVER_LM;
    o->block_cameras = 1;
    o->segment_schedule = 0;
    return DBA_OK;
}

int dba_create(const dba_options *opt, dba_handle **out)
{
    if (!opt || !out) return DBA_E_INVALID_ARG;
    *out = nullptr;
    const dba_options &o = *opt;
    if (o.precision != DBA_PREC_FP64 && o.precision != DBA_PREC_FP32_LOCAL) return DBA_E_INVALID_ARG;
    if (o.loss < 0 || o.loss > 2) return DBA_E_INVALID_ARG;
    if ((o.loss != DBA_LOSS_L2) && !(o.loss_param > 0)) return DBA_E_INVALID_ARG;
    if (!(o.rho_x > 0) || !(o.rho_y > 0)) return DBA_E_INVALID_ARG;
    if (o.lm_steps < 1 || o.lm_steps > 64 || !(o.lm_lambda0 > 0)) return DBA_E_INVALID_ARG;
    if (o.rho_balancing && (!(o.rb_mu > 1) || !(o.rb_tau > 1) || !(o.rho_min > 0) || !(o.rho_max >= o.rho_min)))
        return DBA_E_INVALID_ARG;
    if (o.block_waves != 0 && o.block_waves != 1 && o.block_waves != 2 && o.block_waves != 4 && o.block_waves != 8)
        return DBA_E_INVALID_ARG;
    if (o.persistent < -1 || o.persistent > 1) return DBA_E_INVALID_ARG;
    if (o.start != DBA_START_PLAIN && o.start != DBA_START_LEARNED) return DBA_E_INVALID_ARG;
    if (o.start == DBA_START_LEARNED && o.precision != DBA_PREC_FP32_LOCAL) return DBA_E_INVALID_ARG;
    if (o.learned_lm_steps < 0 || o.learned_lm_steps > 64) return DBA_E_INVALID_ARG;
    if (o.camera_blocks != 0 && o.camera_blocks != 1) return DBA_E_INVALID_ARG;
    if (o.camera_blocks && o.start == DBA_START_LEARNED) return DBA_E_INVALID_ARG;
    if (o.block_points < 0 || o.block_points > dba::kChunk || (o.block_points && !o.camera_blocks))
        return DBA_E_INVALID_ARG;
    if (o.camera_model != DBA_CAMERA_ANGLE_AXIS && o.camera_model != DBA_CAMERA_EULER) return DBA_E_INVALID_ARG;
    if (o.camera_model == DBA_CAMERA_EULER && o.start == DBA_START_LEARNED) return DBA_E_INVALID_ARG;
    if (o.local_solver != DBA_SOLVER_LM && o.local_solver != DBA_SOLVER_GAUSS_NEWTON &&
        o.local_solver != DBA_SOLVER_LBFGS)
        return DBA_E_INVALID_ARG;
    if (o.local_solver != DBA_SOLVER_LM && (o.camera_blocks || o.start == DBA_START_LEARNED))
        return DBA_E_INVALID_ARG;
    if (o.block_cameras != 1 && o.block_cameras != 2) return DBA_E_INVALID_ARG;
    if (o.block_cameras == 2 && !o.camera_blocks) return DBA_E_INVALID_ARG;
    if (o.segment_schedule < 0 || o.segment_schedule > 3) return DBA_E_INVALID_ARG;
    dba_handle *h = new dba_handle();
    h->opt = o;
    h->fp32 = o.precision == DBA_PREC_FP32_LOCAL;
    h->sp.loss = o.loss;
    h->sp.loss_param = o.loss == DBA_LOSS_L2 ? 1.0 : o.loss_param;
    h->sp.lm_steps = o.lm_steps;
    h->sp.lambda0 = o.lm_lambda0;
    h->sp.learned_steps = o.learned_lm_steps;
    h->sp.camera = o.camera_model;
    h->sp.solver = o.local_solver;
    h->start = o.start;
    if (hipSetDevice(o.device) != hipSuccess) {
        delete h;
        return DBA_E_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, o.device) == hipSuccess) h->n_cu = prop.multiProcessorCount;
    if (dba::noalloc_scratch(o.device, &h->noalloc_scratch) != hipSuccess) {
        delete h;
        return DBA_E_DEVICE;
    }
    if (o.stream) {
        h->stream = static_cast<hipStream_t>(o.stream);
    } else {
        if (hipStreamCreate(&h->stream) != hipSuccess) {
            delete h;
            return DBA_E_DEVICE;
        }
        h->own_stream = true;
    }
    h->block_waves = o.block_waves ? o.block_waves : 4;
    h->persistent = o.persistent < 0 ? 0 : o.persistent;
    h->schedule_ready = o.block_waves != 0 && o.persistent >= 0;
    h->seg_sched = o.segment_schedule ? o.segment_schedule : 1;
    h->seg_ready = o.segment_schedule != 0;
    *out = h;
    return DBA_OK;
}

void dba_destroy(dba_handle *h)
{
    if (!h) return;
    (void)hipSetDevice(h->opt.device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    free_set(h);
    free_mlp(h);
    for (hipEvent_t e : h->timing.pool) (void)hipEventDestroy(e);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char *dba_last_error(const dba_handle *h) { return h ? h->err.c_str() : "null handle"; }

int dba_set_problems(dba_handle *h, int32_t np, const dba_problem_desc *probs)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (np < 1 || !probs) return fail(h, DBA_E_INVALID_ARG, "need at least one problem");
    for (int p = 0; p < np; ++p) {
        const int rc = validate(h, p, probs[p]);
        if (rc != DBA_OK) return rc;
    }
    HIP_TRY(h, hipSetDevice(h->opt.device));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    ProblemSet *ps = new ProblemSet();
    const int rc = h->fp32 ? build_set<float>(h, np, probs, ps, ps->a32)
                           : build_set<double>(h, np, probs, ps, ps->a64);
    if (rc != DBA_OK) {
        delete ps;
        return rc;
    }
    free_set(h);
    h->ps = ps;
    h->schedule_ready = h->opt.block_waves != 0 && h->opt.persistent >= 0;
    h->tune_next = 0;
    h->seg_ready = h->opt.segment_schedule != 0;
    h->seg_sched = h->opt.segment_schedule ? h->opt.segment_schedule : 1;
    h->seg_next = 0;
    h->seg_tuned = 0;
    h->seg_ms.clear();
    return DBA_OK;
}

int dba_set_problem(dba_handle *h, int32_t n_cams, int32_t n_points, int64_t n_obs, const int32_t *obs_cam,
                    const int32_t *obs_point, const double *obs_uv, const double *cams, const double *points)
{
    dba_problem_desc d{n_cams, n_points, n_obs, obs_cam, obs_point, obs_uv, cams, points};
    return dba_set_problems(h, 1, &d);
}

int dba_iterate(dba_handle *h, int32_t n_iters)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (!h->ps) return fail(h, DBA_E_STATE, "no problem set");
    if (n_iters < 0) return fail(h, DBA_E_INVALID_ARG, "n_iters < 0");
    if (h->start == DBA_START_LEARNED && !(h->mlp && h->mlp->ready))
        return fail(h, DBA_E_STATE, "learned start without a network (dba_set_mlp or dba_mlp_train)");
    HIP_TRY(h, hipSetDevice(h->opt.device));
    return h->fp32 ? iterate_impl<float>(h, h->ps->a32, n_iters) : iterate_impl<double>(h, h->ps->a64, n_iters);
}

int dba_residuals(dba_handle *h, int32_t p, int32_t want_rmse, dba_residual_report *out)
{
    if (!h || !out) return DBA_E_INVALID_ARG;
    h->err.clear();
    int rc = check_problem(h, p);
    if (rc != DBA_OK) return fail(h, rc, "bad problem index %d", p);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    ProblemSet &ps = *h->ps;
    Ctrl c;
    const Ctrl *dctrl = h->fp32 ? ps.a32.ctrl : ps.a64.ctrl;
    HIP_TRY(h, hipMemcpyAsync(&c, dctrl + p, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    std::memset(out, 0, sizeof(*out));
    double st[dba::kEpart] = {0, 0, 0, 0, 0};
    if (want_rmse) {
        hipError_t e = h->fp32 ? dba::launch_eval<float>(ps.a32, h->sp, h->stream)
                               : dba::launch_eval<double>(ps.a64, h->sp, h->stream);
        HIP_TRY(h, e);
        const double *dst = (h->fp32 ? ps.a32.estats : ps.a64.estats) + (size_t)p * dba::kEpart;
        HIP_TRY(h, hipMemcpyAsync(st, dst, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    out->primal = c.primal;
    out->dual = c.dual;
    out->rho_x = c.last_rho_x;
    out->rho_y = c.last_rho_y;
    out->next_rho_x = c.rho_x;
    out->next_rho_y = c.rho_y;
    out->iteration = c.iteration;
    out->nonfinite = c.nonfinite;
    if (want_rmse) {
        const double L = (double)ps.L[p];
        out->rmse = std::sqrt(st[0] / L);
        out->robust_cost = st[1];
        out->mean_error = st[2] / L;
        out->rmse_masked = st[4] > 0 ? std::sqrt(st[3] / st[4]) : 0.0;
        if (!std::isfinite(st[0])) out->nonfinite = 1;
    }
    return DBA_OK;
}

int dba_set_eval_mask(dba_handle *h, int32_t p, const uint8_t *mask)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    int rc = check_problem(h, p);
    if (rc != DBA_OK) return fail(h, rc, "bad problem index %d", p);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    ProblemSet &ps = *h->ps;
    const ProblemRange &r = ps.ranges[p];
    const long long s0 = (long long)r.chunk0 * dba::kChunk, ns = (long long)r.n_chunks * dba::kChunk;
    std::vector<int> orig(ns), pslot(ns);
    const int *d_orig = h->fp32 ? ps.a32.slot_orig : ps.a64.slot_orig;
    const int *d_pslot = h->fp32 ? ps.a32.pslot : ps.a64.pslot;
    HIP_TRY(h, hipMemcpy(orig.data(), d_orig + s0, ns * sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(h, hipMemcpy(pslot.data(), d_pslot + s0, ns * sizeof(int), hipMemcpyDeviceToHost));
    std::vector<uint8_t> m(ns, 1);
    if (mask)
        for (long long s = 0; s < ns; ++s) m[s] = pslot[s] >= 0 ? (mask[orig[s]] != 0) : 0;
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    HIP_TRY(h, hipMemcpy(ps.mask + s0, m.data(), ns, hipMemcpyHostToDevice));
    return DBA_OK;
}

int dba_get_params(dba_handle *h, int32_t p, double *cams, double *points)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    int rc = check_problem(h, p);
    if (rc != DBA_OK) return fail(h, rc, "bad problem index %d", p);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    ProblemSet &ps = *h->ps;
    const ProblemRange &r = ps.ranges[p];
    std::vector<double> cy((size_t)r.n_cams * dba::kConsY);
    std::vector<double4> cx(r.n_points);
    const double *dcy = h->fp32 ? ps.a32.cons_y : ps.a64.cons_y;
    const double4 *dcx = h->fp32 ? ps.a32.cons_x : ps.a64.cons_x;
    HIP_TRY(h, hipMemcpyAsync(cy.data(), dcy + (size_t)r.cam0 * dba::kConsY, cy.size() * sizeof(double),
                              hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(cx.data(), dcx + r.pt0, cx.size() * sizeof(double4), hipMemcpyDeviceToHost,
                              h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (cams)
        for (int j = 0; j < r.n_cams; ++j)
            for (int c = 0; c < 9; ++c) cams[9 * (size_t)j + c] = cy[(size_t)j * dba::kConsY + c];
    if (points)
        for (int i = 0; i < r.n_points; ++i) {
            points[3 * (size_t)i] = cx[i].x;
            points[3 * (size_t)i + 1] = cx[i].y;
            points[3 * (size_t)i + 2] = cx[i].z;
        }
    return DBA_OK;
}

int dba_get_state(dba_handle *h, int32_t p, double *copies, double *duals)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    int rc = check_problem(h, p);
    if (rc != DBA_OK) return fail(h, rc, "bad problem index %d", p);
    HIP_TRY(h, hipSetDevice(h->opt.device));
    ProblemSet &ps = *h->ps;
    const long long L = ps.L[p];
    double *d = nullptr;
    HIP_TRY(h, hipMalloc(&d, 24 * (size_t)L * sizeof(double)));
    hipError_t e = h->fp32 ? dba::launch_materialize<float>(ps.a32, p, d, d + 12 * L, h->stream)
                           : dba::launch_materialize<double>(ps.a64, p, d, d + 12 * L, h->stream);
    if (e == hipSuccess && copies)
        e = hipMemcpyAsync(copies, d, 12 * L * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && duals)
        e = hipMemcpyAsync(duals, d + 12 * L, 12 * L * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(d);
    HIP_TRY(h, e);
    return DBA_OK;
}

int dba_problem_info(const dba_handle *h, int32_t p, int32_t *m, int32_t *n, int64_t *L)
{
    if (!h) return DBA_E_INVALID_ARG;
    if (!h->ps) return DBA_E_STATE;
    if (p < 0 || p >= h->ps->n_problems) return DBA_E_INVALID_ARG;
    if (m) *m = h->ps->m[p];
    if (n) *n = h->ps->n[p];
    if (L) *L = h->ps->L[p];
    return DBA_OK;
}

int dba_set_kernel_timing(dba_handle *h, int32_t enable)
{
    if (!h) return DBA_E_INVALID_ARG;
    h->err.clear();
    if (enable < 0 || enable > 3) return fail(h, DBA_E_INVALID_ARG, "timing mode %d", enable);
    int rc = collect_timing(h);
    if (rc != DBA_OK) return rc;
    h->timing.on = enable != 0;
    // 1: every kernel; 2: the local solve only (ids 0 and 3); 3: as 2, in
    // the first iteration of each replayed graph only (bit kFirstOnly)
    h->timing.mask = enable == 3 ? (0x9u | kFirstOnly) : enable == 2 ? 0x9u : 0xFu;
    for (int k = 0; k < kKernels; ++k) {
        h->timing.total_ms[k] = 0.0;
        h->timing.launches[k] = 0;
    }
    return DBA_OK;
}

int dba_kernel_times(dba_handle *h, double *total_ms, int64_t *launches)
{
    if (!h || !total_ms || !launches) return DBA_E_INVALID_ARG;
    h->err.clear();
    int rc = collect_timing(h);
    if (rc != DBA_OK) return rc;
    for (int k = 0; k < kKernels; ++k) {
        total_ms[k] = h->timing.total_ms[k];
        launches[k] = h->timing.launches[k];
    }
    return DBA_OK;
}

int dba_schedule(const dba_handle *h, int32_t *bw, int32_t *pers, int32_t *tuned)
{
    if (!h) return DBA_E_INVALID_ARG;
    if (bw) *bw = h->block_waves;
    if (pers) *pers = h->persistent;
    if (tuned) *tuned = h->tuned;
    return DBA_OK;
}

int dba_segment_schedule(const dba_handle *h, int32_t *segment_schedule, int32_t *tuned)
{
    if (!h) return DBA_E_INVALID_ARG;
    if (segment_schedule) *segment_schedule = h->seg_sched;
    if (tuned) *tuned = h->seg_tuned;
    return DBA_OK;
}

}  // extern "C"
