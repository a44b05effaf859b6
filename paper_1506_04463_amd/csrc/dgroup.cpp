// Grouped dense shifted solves (see fh_dgroup.h) and the tile autotuner of
// the grouped complex-FP32 GEMM.
#include <algorithm>
#include <cstring>
#include <functional>

#include "fh_dgroup.h"

namespace fh {

// ---------------------------------------------------------------------------
// autotuner: time the two MFMA tiles on a GEMM of the given shape (C -= A B
// with M x K and K x N operands in scratch memory) and keep the faster one
// per shape class for the life of the handle
// ---------------------------------------------------------------------------
static int autotune_tile(Ctx& c, int M, int N, int K, int copies) {
    auto cls = [](int v) {
        int b = 1;
        while (b < v) b <<= 1;
        return b;
    };
    const std::string key = std::to_string(cls(M)) + "x" + std::to_string(cls(N)) + "x" + std::to_string(K) + "x" +
                            std::to_string(cls(copies));
    auto f = c.tuned.find(key);
    if (f != c.tuned.end()) return f->second;
    const size_t a = (size_t)M * K, b = (size_t)K * N, cc = (size_t)M * N;
    cf* S = (cf*)c.tune_scratch.ensure(sizeof(cf) * (a + b + cc * copies));
    FH_HIP(hipMemsetAsync(S, 0, sizeof(cf) * (a + b + cc * copies), c.stream));
    std::vector<GItem<float>> items;
    for (int q = 0; q < copies; ++q)
        items.push_back(GItem<float>{S, S + a, S + a + b + q * cc, M, N, K, K, N, N, 0, 0, cx(-1.0f, 0.0f), 1});
    hipEvent_t e0, e1;
    FH_HIP(hipEventCreate(&e0));
    FH_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int pick = GTILE_64;
    for (int tile : {GTILE_64, GTILE_32}) {
        GroupPlan<float> plan;
        group_gemm_plan<float>(plan, false, items, tile);
        plan.run(c.stream);   // warm-up
        FH_HIP(hipEventRecord(e0, c.stream));
        for (int r = 0; r < 3; ++r) plan.run(c.stream);
        FH_HIP(hipEventRecord(e1, c.stream));
        FH_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        FH_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            pick = tile;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c.tuned[key] = pick;
    return pick;
}

// ---------------------------------------------------------------------------
void dg_build(Ctx& c, DenseGroup& G, const std::vector<Prob*>& probs,
              const std::vector<std::vector<std::complex<double>>>& zs, bool mixed, fh_report* rep) {
    hipStream_t st = c.stream;
    FH_HIP(hipStreamSynchronize(st));
    G.mixed = mixed;
    G.prob.clear();
    G.n.clear();
    G.z.clear();
    G.moff.clear();
    G.poff.clear();
    size_t mt = 0, pt = 0;
    int nmax = 0;
    for (size_t i = 0; i < probs.size(); ++i)
        for (const auto& zz : zs[i]) {
            G.prob.push_back(probs[i]);
            G.n.push_back(probs[i]->n);
            G.z.push_back(zz);
            G.moff.push_back(mt);
            G.poff.push_back(pt);
            mt += (size_t)probs[i]->n * probs[i]->n;
            pt += probs[i]->n;
            nmax = std::max(nmax, probs[i]->n);
        }
    G.count = (int)G.n.size();
    const int cnt = G.count;
    std::vector<zd> hz(cnt), hzc(cnt);
    for (int s = 0; s < cnt; ++s) {
        hz[s] = zd{G.z[s].real(), G.z[s].imag()};
        hzc[s] = zd{G.z[s].real(), -G.z[s].imag()};
    }
    zd* dz = (zd*)G.dz.ensure(sizeof(zd) * cnt);
    zd* dzc = (zd*)G.dzc.ensure(sizeof(zd) * cnt);
    FH_HIP(hipMemcpy(dz, hz.data(), sizeof(zd) * cnt, hipMemcpyHostToDevice));
    FH_HIP(hipMemcpy(dzc, hzc.data(), sizeof(zd) * cnt, hipMemcpyHostToDevice));
    zd* M64 = (zd*)G.M64.ensure(sizeof(zd) * mt);
    int* ipiv = (int*)G.ipiv.ensure(sizeof(int) * pt);
    int* info = (int*)G.info.ensure(sizeof(int) * cnt);
    // M_s = z_s B - A, problem by problem (its nodes are consecutive)
    for (int s = 0; s < cnt;) {
        Prob* p = G.prob[s];
        int e = s;
        while (e < cnt && G.prob[e] == p) ++e;
        form_shift(st, p->n, (const zd*)p->A.val, p->A.ld, p->hasB ? (const zd*)p->B.val : nullptr, p->B.ld, e - s,
                   dz + s, M64 + G.moff[s]);
        s = e;
    }
    std::vector<int*> pv(cnt), iv(cnt);
    for (int s = 0; s < cnt; ++s) {
        pv[s] = ipiv + G.poff[s];
        iv[s] = info + s;
    }
    if (mixed) {
        G.tile_lu = autotune_tile(c, std::max(1, nmax - GNB), std::max(1, nmax - GNB), GNB, std::min(cnt, 8));
        cf* M32 = (cf*)G.M32.ensure(sizeof(cf) * mt);
        cast<float, double>(st, (long)mt, M64, M32);
        std::vector<cf*> mp(cnt);
        for (int s = 0; s < cnt; ++s) mp[s] = M32 + G.moff[s];
        GroupPlan<float> lu;
        group_lu_plan<float>(lu, cnt, mp.data(), G.n.data(), pv.data(), iv.data(), G.tile_lu);
        lu.run(st);
        G.M64.release();   // the FP64 matrices are not kept: residuals use A and B
        // inverses of the complex-FP32 factorizations: LU X = I, n right-hand sides
        cf* inv = (cf*)G.Inv32.ensure(sizeof(cf) * mt);
        FH_HIP(hipMemsetAsync(inv, 0, sizeof(cf) * mt, st));
        long* doffm = (long*)G.doff.ensure(sizeof(long) * cnt);
        int* dnm = (int*)G.dn.ensure(sizeof(int) * cnt);
        FH_HIP(hipMemcpyAsync(doffm, G.moff.data(), sizeof(long) * cnt, hipMemcpyHostToDevice, st));
        FH_HIP(hipMemcpyAsync(dnm, G.n.data(), sizeof(int) * cnt, hipMemcpyHostToDevice, st));
        set_identity(st, cnt, nmax, doffm, dnm, inv);
        std::vector<cf*> xp(cnt);
        for (int s = 0; s < cnt; ++s) xp[s] = inv + G.moff[s];
        GroupPlan<float> sol;
        group_solve_plan<float>(sol, 'N', cnt, mp.data(), G.n.data(), pv.data(), xp.data(), G.n.data(), G.tile_lu);
        sol.run(st);
        FH_HIP(hipStreamSynchronize(st));       // the layout arrays are rewritten by dg_layout
        G.layout_vtot = -1;
        G.M32.release();
    } else {
        std::vector<zd*> mp(cnt);
        for (int s = 0; s < cnt; ++s) mp[s] = M64 + G.moff[s];
        GroupPlan<double> lu;
        group_lu_plan<double>(lu, cnt, mp.data(), G.n.data(), pv.data(), iv.data(), GTILE_64);
        lu.run(st);
    }
    std::vector<int> hinfo(cnt);
    FH_HIP(hipMemcpyAsync(hinfo.data(), info, sizeof(int) * cnt, hipMemcpyDeviceToHost, st));
    FH_HIP(hipStreamSynchronize(st));
    if (rep) rep->n_factor += cnt;
    for (int s = 0; s < cnt; ++s)
        if (hinfo[s] != 0) {
            if (rep) rep->bad_node = s;
            throw Error(FH_SINGULAR_SHIFT, "zero pivot in the LU of (z B - A) of grouped system " + std::to_string(s));
        }
    G.layout_vtot = -1;   // plans point at the factors: rebuild
    G.drop_graphs();
}

void dg_layout(Ctx& c, DenseGroup& G, const std::vector<int>& m) {
    const int cnt = G.count;
    FH_REQUIRE((int)m.size() == cnt, -1, "grouped solve: one column count per system");
    const bool same_m = (G.m == m);
    G.m = m;
    G.voff.assign(cnt, 0);
    long tot = 0;
    int mmax = 0, maxlen = 0;
    for (int s = 0; s < cnt; ++s) {
        G.voff[s] = tot;
        tot += (long)G.n[s] * m[s];
        mmax = std::max(mmax, m[s]);
        maxlen = std::max(maxlen, G.n[s] * m[s]);
    }
    G.vtot = tot;
    G.mmax = mmax;
    G.maxlen = maxlen;
    const size_t vb = sizeof(zd) * std::max<long>(1, tot);
    zd* Xv = (zd*)G.Xv.ensure(vb);
    zd* Xhv = (zd*)G.Xhv.ensure(vb);
    G.Bv.ensure(vb);
    G.Bhv.ensure(vb);
    cf* X32 = nullptr;
    cf* Xh32 = nullptr;
    zd* R = nullptr;
    zd* Rh = nullptr;
    cf* T32 = nullptr;
    cf* Th32 = nullptr;
    if (G.mixed) {
        X32 = (cf*)G.X32.ensure(sizeof(cf) * std::max<long>(1, tot));
        Xh32 = (cf*)G.Xh32.ensure(sizeof(cf) * std::max<long>(1, tot));
        T32 = (cf*)G.T32.ensure(sizeof(cf) * std::max<long>(1, tot));
        Th32 = (cf*)G.Th32.ensure(sizeof(cf) * std::max<long>(1, tot));
        R = (zd*)G.R.ensure(vb);
        Rh = (zd*)G.Rh.ensure(vb);
    }
    const void* key[5] = {Xv, Xhv, G.mixed ? (const void*)X32 : nullptr, G.mixed ? (const void*)R : nullptr,
                          G.mixed ? (const void*)T32 : nullptr};
    bool same = G.layout_vtot == tot && same_m;
    for (int q = 0; q < 5; ++q) same = same && key[q] == G.layout_key[q];
    if (same) return;
    FH_HIP(hipStreamSynchronize(c.stream));   // earlier solves may still read the old plans
    G.drop_graphs();
    // device layout arrays
    std::vector<int> len(cnt);
    for (int s = 0; s < cnt; ++s) len[s] = G.n[s] * m[s];
    FH_HIP(hipMemcpy(G.doff.ensure(sizeof(long) * cnt), G.voff.data(), sizeof(long) * cnt, hipMemcpyHostToDevice));
    FH_HIP(hipMemcpy(G.dlen.ensure(sizeof(int) * cnt), len.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
    FH_HIP(hipMemcpy(G.dn.ensure(sizeof(int) * cnt), G.n.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
    FH_HIP(hipMemcpy(G.dm.ensure(sizeof(int) * cnt), m.data(), sizeof(int) * cnt, hipMemcpyHostToDevice));
    std::vector<int*> pv(cnt);
    for (int s = 0; s < cnt; ++s) pv[s] = (int*)G.ipiv.p + G.poff[s];
    if (!G.mixed) {
        std::vector<zd*> mp(cnt), xr(cnt), xl(cnt);
        for (int s = 0; s < cnt; ++s) {
            mp[s] = (zd*)G.M64.p + G.moff[s];
            xr[s] = Xv + G.voff[s];
            xl[s] = Xhv + G.voff[s];
        }
        group_solve_plan<double>(G.sN64, 'N', cnt, mp.data(), G.n.data(), pv.data(), xr.data(), m.data(), GTILE_64);
        group_solve_plan<double>(G.sC64, 'C', cnt, mp.data(), G.n.data(), pv.data(), xl.data(), m.data(), GTILE_64);
    } else {
        int nmax = 0;
        for (int v : G.n) nmax = std::max(nmax, v);
        G.tile_solve = autotune_tile(c, nmax, std::max(1, mmax), nmax, std::min(cnt, 8));
        // solves: X32 = M^{-1} T32 (right), Xh32 = M^{-H} Th32 (left)
        std::vector<GItem<float>> gr, gl;
        for (int s = 0; s < cnt; ++s) {
            if (m[s] <= 0) continue;
            const int n = G.n[s];
            const cf* inv = (const cf*)G.Inv32.p + G.moff[s];
            gr.push_back(GItem<float>{inv, T32 + G.voff[s], X32 + G.voff[s], n, m[s], n, n, m[s], m[s], 0, 0,
                                      cx(1.0f, 0.0f), 0});
            gl.push_back(GItem<float>{inv, Th32 + G.voff[s], Xh32 + G.voff[s], n, m[s], n, n, m[s], m[s], 0, 0,
                                      cx(1.0f, 0.0f), 0});
        }
        group_gemm_plan<float>(G.sN32, false, gr, G.tile_solve);
        group_gemm_plan<float>(G.sC32, true, gl, G.tile_solve);
        // FP64 residual products: R_s += A X_s, Rh_s += A^H Xh_s, and the B terms
        std::vector<GItem<double>> iN, iC, bN, bC;
        for (int s = 0; s < cnt; ++s) {
            if (m[s] <= 0) continue;
            Prob* p = G.prob[s];
            const int n = G.n[s];
            const zd* A = (const zd*)p->A.val;
            iN.push_back(GItem<double>{A, Xv + G.voff[s], R + G.voff[s], n, m[s], n, (int)p->A.ld, m[s], m[s], 0, 0,
                                       cx(1.0, 0.0), 1});
            iC.push_back(GItem<double>{A, Xhv + G.voff[s], Rh + G.voff[s], n, m[s], n, (int)p->A.ld, m[s], m[s], 0, 0,
                                       cx(1.0, 0.0), 1});
            if (p->hasB) {
                const zd* Bm = (const zd*)p->B.val;
                const std::complex<double> zz = G.z[s];
                bN.push_back(GItem<double>{Bm, Xv + G.voff[s], R + G.voff[s], n, m[s], n, (int)p->B.ld, m[s], m[s], 0,
                                           0, cx(-zz.real(), -zz.imag()), 1});
                bC.push_back(GItem<double>{Bm, Xhv + G.voff[s], Rh + G.voff[s], n, m[s], n, (int)p->B.ld, m[s], m[s],
                                           0, 0, cx(-zz.real(), zz.imag()), 1});
            }
        }
        group_gemm_plan<double>(G.resN, false, iN, GTILE_64);
        group_gemm_plan<double>(G.resC, true, iC, GTILE_64);
        group_gemm_plan<double>(G.resBN, false, bN, GTILE_64);
        group_gemm_plan<double>(G.resBC, true, bC, GTILE_64);
    }
    for (int q = 0; q < 5; ++q) G.layout_key[q] = key[q];
    G.layout_vtot = tot;
}

void dg_destroy(DenseGroup* g) { delete g; }

// complex-FP32 dense contour filter of one problem: the grouped engine with
// one system per node, factors kept across calls for the same nodes
void dense_filter_group(Ctx& c, Prob& p, int ne, const cplx* z, const cplx* w, int m0, const zd* Y, const zd* Yh,
                        zd* Q, zd* Qh, const fh_opts& o, fh_report* rep) {
    hipStream_t st = c.stream;
    if (!p.dg) p.dg = new DenseGroup();
    DenseGroup& G = *p.dg;
    bool reuse = o.save_factors && G.mixed && G.count == ne;
    for (int j = 0; reuse && j < ne; ++j) reuse = G.z[j] == z[j];
    if (!reuse) dg_build(c, G, {&p}, {std::vector<cplx>(z, z + ne)}, true, rep);
    dg_layout(c, G, std::vector<int>(ne, m0));
    const long blk = (long)p.n * m0;
    zd* T = (zd*)c.fb.R.ensure(sizeof(zd) * blk);
    apply_B(c, p, 0, m0, Y, T);
    replicate<double>(st, blk, T, (zd*)G.Bv.p, ne);
    apply_B(c, p, 1, m0, Yh, T);
    replicate<double>(st, blk, T, (zd*)G.Bhv.p, ne);
    dg_solve(c, G, o, rep);
    zd* wd = (zd*)c.fb.wdev.ensure(sizeof(zd) * ne);
    FH_HIP(hipMemcpyAsync(wd, w, sizeof(zd) * ne, hipMemcpyHostToDevice, st));
    accumulate(st, ne, blk, (const zd*)G.Xv.p, blk, wd, false, Q);
    accumulate(st, ne, blk, (const zd*)G.Xhv.p, blk, wd, true, Qh);
    FH_HIP(hipStreamSynchronize(st));
}

// Run body(stream) through a HIP graph: captured on the handle's capture
// stream the first time (profiling off meanwhile), replayed afterwards, and
// ordered after / before the work of the handle's stream by events.
static void run_graph(Ctx& c, hipGraphExec_t& exec, const std::function<void(hipStream_t)>& body) {
    if (!c.gstream) {
        FH_HIP(hipStreamCreateWithFlags(&c.gstream, hipStreamNonBlocking));
        FH_HIP(hipEventCreateWithFlags(&c.gev[0], hipEventDisableTiming));
        FH_HIP(hipEventCreateWithFlags(&c.gev[1], hipEventDisableTiming));
    }
    if (!exec) {
        Prof* saved = tl_prof();
        tl_prof() = nullptr;
        FH_HIP(hipStreamBeginCapture(c.gstream, hipStreamCaptureModeThreadLocal));
        hipGraph_t g = nullptr;
        try {
            body(c.gstream);
        } catch (...) {
            (void)hipStreamEndCapture(c.gstream, &g);
            if (g) (void)hipGraphDestroy(g);
            tl_prof() = saved;
            throw;
        }
        FH_HIP(hipStreamEndCapture(c.gstream, &g));
        tl_prof() = saved;
        const hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        FH_HIP(e);
    }
    FH_HIP(hipEventRecord(c.gev[0], c.stream));
    FH_HIP(hipStreamWaitEvent(c.gstream, c.gev[0], 0));
    FH_HIP(hipGraphLaunch(exec, c.gstream));
    FH_HIP(hipEventRecord(c.gev[1], c.gstream));
    FH_HIP(hipStreamWaitEvent(c.stream, c.gev[1], 0));
}

// FP64 fallback of a complex-FP32 group: the systems `bad` (whose FP32
// refinement stalled above the inner tolerance: a node so close to an
// eigenvalue that cond(z B - A) u_32 approaches 1) are factored in FP64 (once,
// while the set stays the same) and solved directly; their solutions replace
// the refined ones in G.Xv / G.Xhv.
static void dg_fp64_fallback(Ctx& c, DenseGroup& G, const std::vector<int>& bad, const fh_opts& o) {
    hipStream_t st = c.stream;
    if (!G.fb64 || G.fb_sys != bad) {
        G.fb64.reset(new DenseGroup());
        std::vector<Prob*> probs;
        std::vector<std::vector<std::complex<double>>> zs;
        for (int s : bad) {
            if (probs.empty() || probs.back() != G.prob[s]) {
                probs.push_back(G.prob[s]);
                zs.emplace_back();
            }
            zs.back().push_back(G.z[s]);
        }
        dg_build(c, *G.fb64, probs, zs, false, nullptr);
        G.fb_sys = bad;
    }
    DenseGroup& F = *G.fb64;
    std::vector<int> m(bad.size());
    for (size_t k = 0; k < bad.size(); ++k) m[k] = G.m[bad[k]];
    dg_layout(c, F, m);
    for (size_t k = 0; k < bad.size(); ++k) {
        const int s = bad[k];
        const size_t bytes = sizeof(zd) * (size_t)G.n[s] * G.m[s];
        FH_HIP(hipMemcpyAsync((zd*)F.Bv.p + F.voff[k], (const zd*)G.Bv.p + G.voff[s], bytes, hipMemcpyDeviceToDevice, st));
        FH_HIP(hipMemcpyAsync((zd*)F.Bhv.p + F.voff[k], (const zd*)G.Bhv.p + G.voff[s], bytes, hipMemcpyDeviceToDevice,
                              st));
    }
    dg_solve(c, F, o, nullptr);
    for (size_t k = 0; k < bad.size(); ++k) {
        const int s = bad[k];
        const size_t bytes = sizeof(zd) * (size_t)G.n[s] * G.m[s];
        FH_HIP(hipMemcpyAsync((zd*)G.Xv.p + G.voff[s], (const zd*)F.Xv.p + F.voff[k], bytes, hipMemcpyDeviceToDevice, st));
        FH_HIP(hipMemcpyAsync((zd*)G.Xhv.p + G.voff[s], (const zd*)F.Xhv.p + F.voff[k], bytes, hipMemcpyDeviceToDevice,
                              st));
    }
}

double dg_solve(Ctx& c, DenseGroup& G, const fh_opts& o, fh_report* rep) {
    const long tot = G.vtot;
    const int cnt = G.count;
    zd* Bv = (zd*)G.Bv.p;
    zd* Bhv = (zd*)G.Bhv.p;
    zd* Xv = (zd*)G.Xv.p;
    zd* Xhv = (zd*)G.Xhv.p;
    if (rep) rep->n_solve += 2 * cnt;
    if (!G.mixed) {
        auto body = [&](hipStream_t st) {
            FH_HIP(hipMemcpyAsync(Xv, Bv, sizeof(zd) * tot, hipMemcpyDeviceToDevice, st));
            FH_HIP(hipMemcpyAsync(Xhv, Bhv, sizeof(zd) * tot, hipMemcpyDeviceToDevice, st));
            G.sN64.run(st);
            G.sC64.run(st);
        };
        if (o.graph) run_graph(c, G.g_fp64, body);
        else body(c.stream);
        return 0.0;
    }
    hipStream_t st0 = c.stream;
    cf* X32 = (cf*)G.X32.p;
    cf* Xh32 = (cf*)G.Xh32.p;
    cf* T32 = (cf*)G.T32.p;
    cf* Th32 = (cf*)G.Th32.p;
    zd* R = (zd*)G.R.p;
    zd* Rh = (zd*)G.Rh.p;
    const long* off = (const long*)G.doff.p;
    const int* len = (const int*)G.dlen.p;
    const int* dn = (const int*)G.dn.p;
    const int* dm = (const int*)G.dm.p;
    const int C = cnt * G.mmax;
    double* nrm = (double*)G.nrm.ensure(sizeof(double) * 4 * (size_t)std::max(1, C));
    // shifts of the residual initialisation R = B - z X: zero for systems whose
    // B term comes from a GEMM (a problem with B), z / conj(z) otherwise
    std::vector<zd> hz0(2 * (size_t)cnt);
    for (int s = 0; s < cnt; ++s) {
        const bool b = G.prob[s]->hasB;
        hz0[s] = b ? zd{0.0, 0.0} : zd{G.z[s].real(), G.z[s].imag()};
        hz0[cnt + s] = b ? zd{0.0, 0.0} : zd{G.z[s].real(), -G.z[s].imag()};
    }
    zd* zr = (zd*)G.zb.ensure(sizeof(zd) * 2 * cnt);
    const zd* zl = zr + cnt;
    FH_HIP(hipMemcpyAsync(zr, hz0.data(), sizeof(zd) * 2 * cnt, hipMemcpyHostToDevice, st0));
    set_colnorm(st0, cnt, G.mmax, off, dn, dm, Bv, nrm);
    set_colnorm(st0, cnt, G.mmax, off, dn, dm, Bhv, nrm + C);
    std::vector<double> hb(2 * (size_t)C), hr(2 * (size_t)C), h1;
    FH_HIP(hipMemcpyAsync(hb.data(), nrm, sizeof(double) * 2 * C, hipMemcpyDeviceToHost, st0));
    // one refinement step: d = LU32^{-1} r in complex FP32, x += d, r = b - (z B - A) x in FP64
    auto body = [&](hipStream_t st, bool first) {
        cast<float, double>(st, tot, first ? Bv : R, T32);
        cast<float, double>(st, tot, first ? Bhv : Rh, Th32);
        G.sN32.run(st);
        G.sC32.run(st);
        if (first) {
            cast<double, float>(st, tot, X32, Xv);
            cast<double, float>(st, tot, Xh32, Xhv);
        } else {
            add_cast(st, tot, X32, Xv);
            add_cast(st, tot, Xh32, Xhv);
        }
        set_resid_init(st, cnt, G.maxlen, off, len, zr, Bv, Xv, R);
        set_resid_init(st, cnt, G.maxlen, off, len, zl, Bhv, Xhv, Rh);
        G.resBN.run(st);
        G.resBC.run(st);
        G.resN.run(st);
        G.resC.run(st);
        set_colnorm(st, cnt, G.mmax, off, dn, dm, R, nrm + 2 * C);
        set_colnorm(st, cnt, G.mmax, off, dn, dm, Rh, nrm + 3 * C);
    };
    double worst = 0.0;
    const int steps = std::max(1, o.max_refine);
    for (int it = 0; it < steps; ++it) {
        const bool first = (it == 0);
        if (o.graph) run_graph(c, first ? G.g_first : G.g_next, [&](hipStream_t st) { body(st, first); });
        else body(st0, first);
        FH_HIP(hipMemcpyAsync(hr.data(), nrm + 2 * C, sizeof(double) * 2 * C, hipMemcpyDeviceToHost, st0));
        FH_HIP(hipStreamSynchronize(st0));
        const double prev = worst;
        worst = 0.0;
        for (int q = 0; q < 2 * C; ++q) worst = std::max(worst, hb[q] > 0 ? hr[q] / hb[q] : 0.0);
        if (first) h1 = hr;
        if (rep) rep->inner_steps += 1;
        if (!(worst > o.inner_tol)) break;
        // stop at the FP64 rounding floor: a step that does not halve the residual
        if (it > 0 && !(worst < 0.5 * prev)) break;
    }
    if (steps > 1 && worst > o.inner_tol) {
        // the refinement ended (stalled, or out of steps) above the
        // tolerance: systems still above it that gained less than a factor of
        // 1,000 over their first complex-FP32 solve (the FP32 factors contract
        // slowly or not at all; a system that reached its FP64 rounding floor
        // has gained far more) get FP64 factors.  A single refinement step
        // (max_refine = 1) asks for the plain FP32 solve and never falls back.
        std::vector<int> bad;
        double rest = 0.0;
        for (int s = 0; s < cnt; ++s) {
            double rs = 0.0, r1 = 0.0;
            for (int col = 0; col < G.m[s]; ++col)
                for (int side = 0; side < 2; ++side) {
                    const int q = side * C + s * G.mmax + col;
                    rs = std::max(rs, hb[q] > 0 ? hr[q] / hb[q] : 0.0);
                    r1 = std::max(r1, hb[q] > 0 ? h1[q] / hb[q] : 0.0);
                }
            if (rs > o.inner_tol && rs > 1e-3 * r1) bad.push_back(s);
            else rest = std::max(rest, rs);
        }
        if (!bad.empty()) {
            dg_fp64_fallback(c, G, bad, o);
            if (rep) rep->n_fallback += (long long)bad.size();
            worst = rest;   // the FP64 solves are direct
        }
    }
    if (rep) rep->inner_relres = worst;
    return worst;
}

}  // namespace fh
