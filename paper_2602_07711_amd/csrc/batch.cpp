// Batched (F)GMRES over many right-hand sides and/or independent problems of uneven size: per-problem
// descriptors and work buffers, block/tile offset tables for the grouped launches, and the restart-cycle
// hipGraph (captured once, replayed until every problem is done).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "helm_internal.h"

using namespace helm;


struct helm_batch {
    std::vector<helm_ctx *> ctxs;
    int np = 0, m = 0, fp32 = 0, order = 0, device = 0;
    hipStream_t stream = nullptr;        // private stream (capturable)
    hipStream_t user = nullptr;          // stream of contexts[0]
    std::vector<BProb> hP;
    BProb *dP = nullptr;
    BState *dst = nullptr;
    BParams *dprm = nullptr;
    BLaunch L{};
    std::vector<void *> allocs;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev = nullptr;
    std::string err;
};

namespace {

template <typename T> hipError_t balloc(helm_batch &b, T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T));
    if (e == hipSuccess) {
        b.allocs.push_back(q);
        *p = (T *)q;
    }
    return e;
}

void batch_free(helm_batch *b) {
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    for (void *p : b->allocs) hipFree(p);
    if (b->ev) hipEventDestroy(b->ev);
    if (b->stream) hipStreamDestroy(b->stream);
    delete b;
}

thread_local std::string g_batch_err;

}  // namespace

extern "C" {

helm_status helm_batch_create(helm_batch **out, helm_ctx *const *ctxs, int np, int m, int prec_fp32) {
    g_batch_err.clear();
    if (!out || !ctxs || np < 1 || m < 1 || m > 128) {
        g_batch_err = "invalid batch arguments (np >= 1, 1 <= m <= 128)";
        return HELM_EINVAL;
    }
    *out = nullptr;
    for (int p = 0; p < np; ++p)
        if (!ctxs[p]) { g_batch_err = "NULL context"; return HELM_EINVAL; }
    const int order = ctxs[0]->c.order;
    int dev = 0;
    hipGetDevice(&dev);
    for (int p = 0; p < np; ++p) {
        if (ctxs[p]->c.order != order) { g_batch_err = "all problems of a batch need the same order"; return HELM_EINVAL; }
        if (ctxs[p]->c.device != dev) { g_batch_err = "all contexts must live on the current device"; return HELM_EINVAL; }
        if (ctxs[p]->c.k2i) { g_batch_err = "batched solves take real k^2 only"; return HELM_EUNSUPPORTED; }
        if (ctxs[p]->c.bc_kind == HELM_BC_ABC3) { g_batch_err = "batched solves take the two-point closure"; return HELM_EUNSUPPORTED; }
    }
    helm_batch *b = new helm_batch();
    b->ctxs.assign(ctxs, ctxs + np);
    b->np = np;
    b->m = m;
    b->fp32 = prec_fp32 ? 1 : 0;
    b->order = order;
    b->device = dev;
    b->user = ctxs[0]->c.stream;
    auto fail = [&](helm_status s, const std::string &msg) {
        g_batch_err = msg;
        batch_free(b);
        return s;
    };
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return fail(HELM_EDEVICE, "stream");
    if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) return fail(HELM_EDEVICE, "event");
    const size_t esz = b->fp32 ? sizeof(float2) : sizeof(double2);

    // tile configurations tuned for the first context (helm_autotune), used for every problem of the batch
    // (roles: x forward, y forward, y inverse, x inverse)
    const Ctx &c0 = ctxs[0]->c;
    const int kx = b->fp32 ? 2 : 0, ky = b->fp32 ? 3 : 1;
    const int rcfg[4] = {c0.gemm_cfg[kx], c0.gemm_cfg[ky], c0.gemm_cfg_inv[ky], c0.gemm_cfg_inv[kx]};
    int bm[4], bn[4];
    for (int r = 0; r < 4; ++r) gemm_cfg_tile(rcfg[r], bm[r], bn[r]);
    // z-solve block shape: 16 lines x the largest problem's chunk count (at most 1024 threads)
    int tri_pb = 1;
    for (int p = 0; p < np; ++p) tri_pb = std::max(tri_pb, tri_chunks(ctxs[p]->c.nz));
    if (tri_pb > 1024) return fail(HELM_EUNSUPPORTED, "z-extent too large for the partitioned z-solve");
    int tri_lx = 16;
    while (tri_lx > 1 && tri_lx * tri_pb > 1024) tri_lx /= 2;
    // per-problem descriptors, work buffers and launch offsets
    long long tot_blocks_mv_target = 32768 / STENCIL_TY;   // about 32768 waves over all problems
    std::vector<int> omv(1, 0), otri(1, 0), odot(1, 0), olc(1, 0);
    std::vector<long long> og[4];
    for (auto &v : og) v.assign(1, 0);
    b->hP.resize(np);
    for (int p = 0; p < np; ++p) {
        Ctx &c = ctxs[p]->c;
        BProb &q = b->hP[p];
        q.sp = c.sp;
        // z-chunking for the batch: about tot_blocks_mv_target matvec blocks over all problems
        {
            int txy = q.sp.tiles_x * q.sp.tiles_y;
            long long want = std::max<long long>(1, tot_blocks_mv_target / np / txy);
            want = std::min<long long>(want, c.nz);
            q.sp.zchunk = (int)((c.nz + want - 1) / want);
            q.sp.zchunks = (c.nz + q.sp.zchunk - 1) / q.sp.zchunk;
        }
        q.k2 = c.k2;
        q.fld = c.fld;
        if (b->fp32) {
            q.xfs = c.fx32.fs; q.xfa = c.fx32.fa; q.xis = c.fx32.is; q.xia = c.fx32.ia;
            q.yfs = c.fy32.fs; q.yfa = c.fy32.fa; q.yis = c.fy32.is; q.yia = c.fy32.ia;
        } else {
            q.xfs = c.fx64.fs; q.xfa = c.fx64.fa; q.xis = c.fx64.is; q.xia = c.fx64.ia;
            q.yfs = c.fy64.fs; q.yfa = c.fy64.fa; q.yis = c.fy64.is; q.yia = c.fy64.ia;
        }
        q.dxe = c.dxe;
        q.dye = c.dye;
        q.ax = c.ax; q.ay = c.ay; q.c0 = c.c0; q.hz2 = c.hz * c.hz;
        q.gz = make_double2(c.gamma[2].real(), c.gamma[2].imag());
        q.fx = FoldDesc{c.nx, c.nx - c.nx / 2, c.nx / 2, c.ny * c.nz, c.nx, 0, 1, c.nx - c.nx / 2, 1};
        q.fy = FoldDesc{c.ny, c.ny - c.ny / 2, c.ny / 2, c.nx, c.nx, (long long)c.nx * c.ny, c.nz, c.ny - c.ny / 2, 1};
        q.n = c.n;
        q.nx = c.nx; q.ny = c.ny; q.nz = c.nz;
        q.nblk_dots = dots_blocks(c.n);
        void *zb = nullptr;
        if (balloc(*b, &q.V, (size_t)(m + 1) * c.n) != hipSuccess || hipMalloc(&zb, esz * m * c.n) != hipSuccess)
            return fail(HELM_ENOMEM, "Krylov workspace allocation failed");
        b->allocs.push_back(zb);
        q.Z = zb;
        void *t1 = nullptr, *t2 = nullptr;
        if (hipMalloc(&t1, esz * c.n) != hipSuccess) return fail(HELM_ENOMEM, "work allocation failed");
        b->allocs.push_back(t1);
        if (hipMalloc(&t2, esz * c.n) != hipSuccess) return fail(HELM_ENOMEM, "work allocation failed");
        b->allocs.push_back(t2);
        q.t1 = t1; q.t2 = t2;
        if (ctx_tri_pivots(c) != HELM_OK) return fail(HELM_EDEVICE, "z-solve pivots: " + c.err);
        q.tpiv = c.tpiv_eig.d;
        q.tpiv32 = c.tpiv_eig.f;
        if (balloc(*b, &q.part, (size_t)q.nblk_dots * (m + 2)) != hipSuccess) return fail(HELM_ENOMEM, "partials");
        q.x = nullptr;
        q.F = nullptr;
        int T = q.sp.tiles_x * q.sp.tiles_y * q.sp.zchunks;
        omv.push_back(omv.back() + 8 * ((T + 7) / 8));
        otri.push_back(otri.back() + (int)(((long long)c.nx * c.ny + tri_lx - 1) / tri_lx));
        odot.push_back(odot.back() + q.nblk_dots);
        olc.push_back(olc.back() + (int)((c.n + 1023) / 1024));
        og[0].push_back(og[0].back() + fold_tile_count(FOLD_XF, q.fx, bm[0], bn[0]));
        og[1].push_back(og[1].back() + fold_tile_count(FOLD_YF, q.fy, bm[1], bn[1]));
        og[2].push_back(og[2].back() + fold_tile_count(FOLD_YI, q.fy, bm[2], bn[2]));
        og[3].push_back(og[3].back() + fold_tile_count(FOLD_XI, q.fx, bm[3], bn[3]));
    }
    // step-matvec units: consecutive problems of one context share a block (their operator is read once)
    std::vector<int2> units;
    std::vector<int> omvp(1, 0);
    for (int p = 0; p < np; ++p) {
        const bool pair = p + 1 < np && ctxs[p + 1] == ctxs[p];
        units.push_back(make_int2(p, pair ? p + 1 : -1));
        omvp.push_back(omvp.back() + (omv[p + 1] - omv[p]));
        if (pair) ++p;
    }
    BLaunch &L = b->L;
    if (balloc(*b, &b->dP, np) != hipSuccess || balloc(*b, &b->dst, np) != hipSuccess ||
        balloc(*b, &b->dprm, 1) != hipSuccess)
        return fail(HELM_ENOMEM, "descriptor allocation failed");
    if (balloc(*b, &L.a.H, (size_t)np * (m + 1) * m) != hipSuccess || balloc(*b, &L.a.cs, (size_t)np * m) != hipSuccess ||
        balloc(*b, &L.a.sn, (size_t)np * m) != hipSuccess || balloc(*b, &L.a.g, (size_t)np * (m + 1)) != hipSuccess ||
        balloc(*b, &L.a.coef, (size_t)np * (m + 1)) != hipSuccess)
        return fail(HELM_ENOMEM, "state allocation failed");
    int2 *dunits = nullptr;
    if (balloc(*b, &dunits, units.size()) != hipSuccess || balloc(*b, &L.off.mvp, omvp.size()) != hipSuccess)
        return fail(HELM_ENOMEM, "offset allocation failed");
    if (hipMemcpy(dunits, units.data(), units.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.mvp, omvp.data(), omvp.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return fail(HELM_EDEVICE, "offset upload failed");
    L.units = dunits;
    L.nunits = (int)units.size();
    L.tot_mvp = omvp.back();
    if (balloc(*b, &L.off.mv, np + 1) != hipSuccess || balloc(*b, &L.off.tri, np + 1) != hipSuccess ||
        balloc(*b, &L.off.dot, np + 1) != hipSuccess || balloc(*b, &L.off.lc, np + 1) != hipSuccess ||
        balloc(*b, &L.off.g[0], np + 1) != hipSuccess || balloc(*b, &L.off.g[1], np + 1) != hipSuccess ||
        balloc(*b, &L.off.g[2], np + 1) != hipSuccess || balloc(*b, &L.off.g[3], np + 1) != hipSuccess)
        return fail(HELM_ENOMEM, "offset allocation failed");
    if (hipMemcpy(L.off.mv, omv.data(), omv.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.tri, otri.data(), otri.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.dot, odot.data(), odot.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.lc, olc.data(), olc.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.g[0], og[0].data(), og[0].size() * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.g[1], og[1].data(), og[1].size() * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.g[2], og[2].data(), og[2].size() * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L.off.g[3], og[3].data(), og[3].size() * sizeof(long long), hipMemcpyHostToDevice) != hipSuccess)
        return fail(HELM_EDEVICE, "offset upload failed");
    L.P = b->dP;
    L.st = b->dst;
    L.prm = b->dprm;
    L.np = np;
    L.m = m;
    L.order = order;
    L.fp32 = b->fp32;
    for (int r = 0; r < 4; ++r) L.cfg[r] = rcfg[r];
    L.tri_lx = tri_lx;
    L.tri_pb = tri_pb;
    L.tot_mv = omv.back();
    L.tot_tri = otri.back();
    L.tot_dot = odot.back();
    L.tot_lc = olc.back();
    long long gmax = 0;
    for (int r = 0; r < 4; ++r) {
        L.tot_g[r] = og[r].back();
        gmax = std::max(gmax, L.tot_g[r]);
    }
    // persistent GEMM grid: at most 4 workgroups per CU of a 256-CU device, never more than the tiles
    L.gemm_grid = (int)std::max<long long>(1, std::min<long long>(gmax, 1024));
    *out = b;
    return HELM_OK;
}

void helm_batch_destroy(helm_batch *b) { batch_free(b); }

helm_status helm_batch_solve(helm_batch *b, const void *const *F, void *const *x, int x0_given, double rtol,
                             int maxit, int use_graph, helm_solve_info *infos) {
    if (!b) return HELM_EINVAL;
    if (!F || !x || !(rtol > 0.0) || maxit < 1) { b->err = "invalid solve arguments"; return HELM_EINVAL; }
    for (int p = 0; p < b->np; ++p)
        if (!F[p] || !x[p]) { b->err = "NULL vector"; return HELM_EINVAL; }
#define BTRY(expr)                                                                                      \
    do {                                                                                                \
        hipError_t _e = (expr);                                                                         \
        if (_e != hipSuccess) {                                                                         \
            b->err = std::string(#expr) + ": " + hipGetErrorString(_e);                                 \
            return HELM_EDEVICE;                                                                        \
        }                                                                                               \
    } while (0)
    for (int p = 0; p < b->np; ++p) {
        b->hP[p].F = (const double2 *)F[p];
        b->hP[p].x = (double2 *)x[p];
    }
    BParams prm{rtol, maxit, b->m, cgs_reorth()};
    // order after prior work on the caller's stream
    BTRY(hipEventRecord(b->ev, b->user));
    BTRY(hipStreamWaitEvent(b->stream, b->ev, 0));
    BTRY(hipMemcpyAsync(b->dP, b->hP.data(), b->hP.size() * sizeof(BProb), hipMemcpyHostToDevice, b->stream));
    BTRY(hipMemcpyAsync(b->dprm, &prm, sizeof(BParams), hipMemcpyHostToDevice, b->stream));
    BTRY(hipStreamSynchronize(b->stream));
    if (!x0_given) BTRY(bl_zero_x(b->L, b->stream));
    BTRY(bl_init(b->L, b->stream));
    std::vector<BState> hs(b->np);
    auto read_states = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(hs.data(), b->dst, hs.size() * sizeof(BState), hipMemcpyDeviceToHost, b->stream);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(b->stream);
    };
    BTRY(read_states());
    for (int p = 0; p < b->np; ++p)   // F = 0: the solution is 0 whatever the initial guess
        if (hs[p].bnorm == 0.0 && x0_given) BTRY(launch_fill_zero(b->hP[p].x, b->hP[p].n, b->stream));
    if (use_graph && !b->exec) {
        BTRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        hipError_t ce = bl_cycle(b->L, b->stream);
        hipGraph_t g = nullptr;
        hipError_t ee = hipStreamEndCapture(b->stream, &g);
        if (ce != hipSuccess || ee != hipSuccess) {
            if (g) hipGraphDestroy(g);
            b->err = std::string("graph capture failed: ") + hipGetErrorString(ce != hipSuccess ? ce : ee);
            return HELM_EDEVICE;
        }
        b->graph = g;
        BTRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    int guard = 0;
    for (;;) {
        if (use_graph) BTRY(hipGraphLaunch(b->exec, b->stream));
        else BTRY(bl_cycle(b->L, b->stream));
        BTRY(read_states());
        bool all_done = true, all_settled = true;
        for (auto &s : hs) {
            all_done = all_done && s.done;
            // settled: the Givens estimate met rtol or the iteration cap was hit; the restart test confirms
            all_settled = all_settled && (s.done || s.relres_est <= rtol || s.its >= maxit);
        }
        if (all_done) break;
        if (all_settled) {
            BTRY(bl_restart(b->L, b->stream));
            BTRY(read_states());
            all_done = true;
            for (auto &s : hs) all_done = all_done && s.done;
            if (all_done) break;
        }
        if (++guard > maxit + 2) { b->err = "batch did not finish"; return HELM_ENUMERIC; }
    }
    BTRY(hipEventRecord(b->ev, b->stream));
    BTRY(hipStreamWaitEvent(b->user, b->ev, 0));
    bool all_conv = true, nonfinite = false;
    for (int p = 0; p < b->np; ++p) {
        const BState &s = hs[p];
        all_conv = all_conv && s.converged;
        nonfinite = nonfinite || !std::isfinite(s.relres_true);
        if (infos) {
            helm_solve_info inf{};
            inf.iters = s.its;
            inf.restarts = s.cycles;
            inf.converged = s.converged;
            inf.reorths = s.cancel;
            inf.relres_est = s.relres_est;
            inf.relres_true = s.relres_true;
            infos[p] = inf;
        }
    }
    if (nonfinite) { b->err = "non-finite residual in a batched problem"; return HELM_ENUMERIC; }
    if (!all_conv) { b->err = "some problems reached maxit"; return HELM_ENOCONV; }
    return HELM_OK;
#undef BTRY
}

const char *helm_batch_last_error(const helm_batch *b) { return b ? b->err.c_str() : g_batch_err.c_str(); }

}  // extern "C"
