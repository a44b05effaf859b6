// Sparse (CSR) path: symbolic analysis on the host (once per problem), the
// per-node ILU(0) factorizations kept across FEAST iterations, the
// column-batched GMRES(restart) solver with ILU(0) right preconditioning in
// FP64 or in complex FP32 wrapped in FP64 iterative refinement, and the
// contour filter built on it.
//
// The filter can run in its plain form (right-hand sides B Y and B^H Yh, the
// paper's eq:qr / eq:ql) or, when the columns of Y are Ritz vectors with Ritz
// values lam, in the algebraically identical residual form
//   (z B - A)^{-1} B y = y/(z - lam) + (z B - A)^{-1} r/(z - lam),  r = A y - lam B y,
// so that each inner solve only has to resolve the Ritz residual.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <cstdlib>

#include "fh_sparse.h"
#include "fh_net.h"

namespace fh {

static int* dev_ints(SparseState& S, const std::vector<int>& h, hipStream_t st) {
    DBuf* b = new DBuf();
    S.owned.push_back(b);
    int* p = (int*)b->ensure(sizeof(int) * std::max<size_t>(1, h.size()));
    if (!h.empty()) {
        FH_HIP(hipMemcpyAsync(p, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, st));
        FH_HIP(hipStreamSynchronize(st));   // h may be reused or freed by the caller
    }
    return p;
}

// rows grouped by level (ascending row index within a level)
static void level_order(const std::vector<int>& lev, int n, std::vector<int>& ptr, std::vector<int>& rows) {
    int nlev = 0;
    for (int i = 0; i < n; ++i) nlev = std::max(nlev, lev[i] + 1);
    ptr.assign(nlev + 1, 0);
    rows.resize(n);
    for (int i = 0; i < n; ++i) ptr[lev[i] + 1]++;
    for (int l = 0; l < nlev; ++l) ptr[l + 1] += ptr[l];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < n; ++i) rows[fill[lev[i]]++] = i;
}

// Level-packed ELL form of one triangular sweep.  entries(i, cols, pos) lists
// the off-diagonal entries of row i (column, position of its value in the LU
// factor on the M pattern); dpos_of(i) is the pivot position or -1 (unit).
template <typename F, typename D>
static SweepDev build_sweep(SparseState& S, const std::vector<int>& lev, int n, bool conjv, F entries, D dpos_of,
                            hipStream_t st, std::vector<int>* posL) {
    std::vector<int> ptr, rows;
    level_order(lev, n, ptr, rows);
    // blocked-layout positions: the forward L sweep (built first) defines the
    // order, every sweep addresses a row by its position in it
    if (posL->empty()) {
        posL->assign(n, 0);
        for (int t = 0; t < n; ++t) (*posL)[rows[t]] = t;
    }
    std::vector<int> pp(n);
    for (int t = 0; t < n; ++t) pp[t] = (*posL)[rows[t]];
    int K = 0;
    std::vector<int> cols, pos;
    for (int i = 0; i < n; ++i) {
        cols.clear();
        pos.clear();
        entries(i, cols, pos);
        K = std::max(K, (int)cols.size());
    }
    std::vector<int> ecol((size_t)K * n, -1), epos((size_t)K * n, -1), dp;
    bool has_diag = false;
    for (int t = 0; t < n; ++t) {
        cols.clear();
        pos.clear();
        entries(rows[t], cols, pos);
        for (size_t k = 0; k < cols.size(); ++k) {
            ecol[k * n + t] = cols[k];
            epos[k * n + t] = pos[k];
        }
        const int d = dpos_of(rows[t]);
        if (d >= 0) has_diag = true;
        dp.push_back(d);
    }
    SweepDev sw;
    sw.lev_ptr = dev_ints(S, ptr, st);
    sw.rows = dev_ints(S, rows, st);
    sw.ppos = dev_ints(S, pp, st);
    sw.nlev = (int)ptr.size() - 1;
    sw.K = K;
    sw.conj = conjv;
    // dependencies as positions within the previous level (for the LDS ring of
    // the sweep kernel), when every dependency lies in the level just before
    std::vector<int> pos_in_level(n);
    for (int l = 0; l < sw.nlev; ++l) {
        sw.wmax = std::max(sw.wmax, ptr[l + 1] - ptr[l]);
        for (int t = ptr[l]; t < ptr[l + 1]; ++t) pos_in_level[rows[t]] = t - ptr[l];
    }
    std::vector<int> eslot((size_t)K * n, -1);
    bool adjacent = true;
    for (int t = 0; t < n; ++t)
        for (int k = 0; k < K; ++k) {
            const int c = ecol[(size_t)k * n + t];
            if (c < 0) continue;
            if (lev[rows[t]] - lev[c] != 1) adjacent = false;
            eslot[(size_t)k * n + t] = pos_in_level[c];
        }
    sw.adjacent = adjacent;
    if (K > 0) {
        sw.ell_col = dev_ints(S, ecol, st);
        sw.ell_pos = dev_ints(S, epos, st);
        sw.ell_slot = dev_ints(S, eslot, st);
    }
    if (has_diag) sw.dpos = dev_ints(S, dp, st);
    return sw;
}

static LevelsDev levels_dev(SparseState& S, const std::vector<int>& lev, int n, hipStream_t st) {
    int nlev = 0;
    for (int i = 0; i < n; ++i) nlev = std::max(nlev, lev[i] + 1);
    std::vector<int> ptr(nlev + 1, 0), rows(n);
    for (int i = 0; i < n; ++i) ptr[lev[i] + 1]++;
    for (int l = 0; l < nlev; ++l) ptr[l + 1] += ptr[l];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int i = 0; i < n; ++i) rows[fill[lev[i]]++] = i;
    LevelsDev L;
    L.ptr = dev_ints(S, ptr, st);
    L.rows = dev_ints(S, rows, st);
    L.nlev = nlev;
    return L;
}

// transpose of a pattern: returns rowptr/col of P^T and, for each entry of P^T,
// the position of the same entry in P
static void transpose_pattern(int n, const std::vector<int>& rp, const std::vector<int>& ci, std::vector<int>& trp,
                              std::vector<int>& tci, std::vector<int>& tpos) {
    const long nnz = rp[n];
    trp.assign(n + 1, 0);
    for (long p = 0; p < nnz; ++p) trp[ci[p] + 1]++;
    for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
    tci.resize(nnz);
    tpos.resize(nnz);
    std::vector<int> fill(trp.begin(), trp.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int p = rp[i]; p < rp[i + 1]; ++p) {
            const int q = fill[ci[p]]++;
            tci[q] = i;
            tpos[q] = p;
        }
}

// column chunk of the ILU sweeps: FH_ILU_CW64 / FH_ILU_CW32 override the defaults
static void ilu_chunk_defaults(SparseState& S) {
    if (const char* e = std::getenv("FH_ILU_CW64")) S.ilu_cw64 = std::max(1, std::atoi(e));
    if (const char* e = std::getenv("FH_ILU_CW32")) S.ilu_cw32 = std::max(1, std::atoi(e));
}

void sparse_prepare(Ctx& c, Prob& p) {
    hipStream_t st = c.stream;
    SparseState* S = new SparseState();
    p.sp = S;
    const int n = p.n;
    const long nnz = p.A.nnz;
    S->n = n;
    S->nnzA = nnz;
    std::vector<int> rp(n + 1), ci(nnz);
    FH_HIP(hipMemcpyAsync(rp.data(), p.A.rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
    FH_HIP(hipMemcpyAsync(ci.data(), p.A.colind, sizeof(int) * nnz, hipMemcpyDeviceToHost, st));
    FH_HIP(hipStreamSynchronize(st));
    FH_REQUIRE(rp[0] == 0 && rp[n] == nnz, -2, "CSR row pointers must start at 0 and end at nnz");
    for (int i = 0; i < n; ++i) {
        FH_REQUIRE(rp[i + 1] >= rp[i], -2, "CSR row pointers must be non-decreasing");
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            FH_REQUIRE(ci[q] >= 0 && ci[q] < n, -2, "CSR column index out of range");
            if (q > rp[i]) FH_REQUIRE(ci[q] > ci[q - 1], -2, "CSR column indices must be sorted and unique per row");
        }
    }
    // M pattern = A pattern + full diagonal
    std::vector<int> mrp(n + 1, 0), mci, a2m(nnz), mdiag(n);
    mci.reserve(nnz + n);
    for (int i = 0; i < n; ++i) {
        bool placed = false;
        for (int q = rp[i]; q < rp[i + 1]; ++q) {
            if (!placed && ci[q] > i) { mdiag[i] = (int)mci.size(); mci.push_back(i); placed = true; }
            if (ci[q] == i) { mdiag[i] = (int)mci.size(); placed = true; }
            a2m[q] = (int)mci.size();
            mci.push_back(ci[q]);
        }
        if (!placed) { mdiag[i] = (int)mci.size(); mci.push_back(i); }
        mrp[i + 1] = (int)mci.size();
    }
    const long nnzM = (long)mci.size();
    S->nnzM = nnzM;
    std::vector<int> trp, tci, t2m, tdiag(n);
    transpose_pattern(n, mrp, mci, trp, tci, t2m);
    for (int i = 0; i < n; ++i)
        for (int q = trp[i]; q < trp[i + 1]; ++q)
            if (tci[q] == i) tdiag[i] = q;
    // ILU(0) update lists: for each L entry (i,k): pairs (pos(i,j), pos(k,j)) for j > k in both rows
    std::vector<int> uptr(nnzM + 1, 0);
    std::vector<int2> upd;
    std::vector<int> wpos(n, -1);
    for (int i = 0; i < n; ++i) {
        for (int q = mrp[i]; q < mrp[i + 1]; ++q) wpos[mci[q]] = q;
        for (int q = mrp[i]; q < mrp[i + 1]; ++q) {
            uptr[q] = (int)upd.size();
            const int k = mci[q];
            if (k >= i) continue;
            for (int r = mdiag[k] + 1; r < mrp[k + 1]; ++r) {
                const int j = mci[r];
                if (wpos[j] >= 0) upd.push_back(make_int2(wpos[j], r));
            }
        }
        for (int q = mrp[i]; q < mrp[i + 1]; ++q) wpos[mci[q]] = -1;
    }
    uptr[nnzM] = (int)upd.size();
    S->nupd = (long)upd.size();
    // level sets of the four triangular sweeps
    std::vector<int> lev(n);
    for (int i = 0; i < n; ++i) {            // L (forward)
        int l = 0;
        for (int q = mrp[i]; q < mdiag[i]; ++q) l = std::max(l, lev[mci[q]] + 1);
        lev[i] = l;
    }
    S->levL = levels_dev(*S, lev, n, st);
    std::vector<int> posL;
    S->swL = build_sweep(*S, lev, n, false,
        [&](int i, std::vector<int>& c, std::vector<int>& ps) {
            for (int q = mrp[i]; q < mdiag[i]; ++q) { c.push_back(mci[q]); ps.push_back(q); } },
        [&](int) { return -1; }, st, &posL);
    for (int i = n - 1; i >= 0; --i) {       // U (backward)
        int l = 0;
        for (int q = mdiag[i] + 1; q < mrp[i + 1]; ++q) l = std::max(l, lev[mci[q]] + 1);
        lev[i] = l;
    }
    S->levU = levels_dev(*S, lev, n, st);
    S->swU = build_sweep(*S, lev, n, false,
        [&](int i, std::vector<int>& c, std::vector<int>& ps) {
            for (int q = mdiag[i] + 1; q < mrp[i + 1]; ++q) { c.push_back(mci[q]); ps.push_back(q); } },
        [&](int i) { return mdiag[i]; }, st, &posL);
    for (int i = 0; i < n; ++i) {            // U^H: lower part of M^T (forward)
        int l = 0;
        for (int q = trp[i]; q < tdiag[i]; ++q) l = std::max(l, lev[tci[q]] + 1);
        lev[i] = l;
    }
    S->levUT = levels_dev(*S, lev, n, st);
    S->swUT = build_sweep(*S, lev, n, true,
        [&](int i, std::vector<int>& c, std::vector<int>& ps) {
            for (int q = trp[i]; q < tdiag[i]; ++q) { c.push_back(tci[q]); ps.push_back(t2m[q]); } },
        [&](int i) { return mdiag[i]; }, st, &posL);
    for (int i = n - 1; i >= 0; --i) {       // L^H: upper part of M^T (backward)
        int l = 0;
        for (int q = tdiag[i] + 1; q < trp[i + 1]; ++q) l = std::max(l, lev[tci[q]] + 1);
        lev[i] = l;
    }
    S->levLT = levels_dev(*S, lev, n, st);
    S->swLT = build_sweep(*S, lev, n, true,
        [&](int i, std::vector<int>& c, std::vector<int>& ps) {
            for (int q = tdiag[i] + 1; q < trp[i + 1]; ++q) { c.push_back(tci[q]); ps.push_back(t2m[q]); } },
        [&](int) { return -1; }, st, &posL);
    S->mrowptr = dev_ints(*S, mrp, st);
    S->mcol = dev_ints(*S, mci, st);
    S->mdiag = dev_ints(*S, mdiag, st);
    S->a2m = dev_ints(*S, a2m, st);
    S->trowptr = dev_ints(*S, trp, st);
    S->tcol = dev_ints(*S, tci, st);
    S->tdiag = dev_ints(*S, tdiag, st);
    S->t2m = dev_ints(*S, t2m, st);
    S->uptr = dev_ints(*S, uptr, st);
    {
        DBuf* b = new DBuf();
        S->owned.push_back(b);
        S->upd = (int2*)b->ensure(sizeof(int2) * std::max<size_t>(1, upd.size()));
        if (!upd.empty()) {
            FH_HIP(hipMemcpyAsync(S->upd, upd.data(), sizeof(int2) * upd.size(), hipMemcpyHostToDevice, st));
            FH_HIP(hipStreamSynchronize(st));
        }
    }
    // A (user arrays) with an FP32 copy; A^T pattern with FP64/FP32 values
    const bool cplx_vals = (p.A.dtype == FH_C128);
    const size_t vb = cplx_vals ? sizeof(zd) : sizeof(double);
    S->A.rowptr = p.A.rowptr;
    S->A.col = p.A.colind;
    S->A.val64 = p.A.val;
    S->A.complex_vals = cplx_vals;
    S->A.nnz = nnz;
    S->AT.nnz = nnz;
    for (int i = 0; i < n; ++i) S->A.maxrow = std::max(S->A.maxrow, rp[i + 1] - rp[i]);
    S->A.val32 = S->aval32.ensure(vb / 2 * std::max<long>(1, nnz));
    cast_vals(st, nnz, cplx_vals, p.A.val, (void*)S->A.val32);
    std::vector<int> atrp, atci, at2a;
    transpose_pattern(n, rp, ci, atrp, atci, at2a);
    S->AT.rowptr = dev_ints(*S, atrp, st);
    for (int i = 0; i < n; ++i) S->AT.maxrow = std::max(S->AT.maxrow, atrp[i + 1] - atrp[i]);
    S->AT.col = dev_ints(*S, atci, st);
    int* at2a_d = dev_ints(*S, at2a, st);
    S->AT.complex_vals = cplx_vals;
    S->AT.val64 = S->atval64.ensure(vb * std::max<long>(1, nnz));
    gather_vals(st, nnz, cplx_vals, p.A.val, at2a_d, (void*)S->AT.val64);
    S->AT.val32 = S->atval32.ensure(vb / 2 * std::max<long>(1, nnz));
    cast_vals(st, nnz, cplx_vals, S->AT.val64, (void*)S->AT.val32);
    // complex symmetric (A = A^T): the transposed pattern is the pattern and
    // every value equals its transposed partner (checked exactly)
    S->csym = atrp == rp && atci == ci;
    if (S->csym && nnz > 0) {
        std::vector<double> hv(nnz * (cplx_vals ? 2 : 1));
        FH_HIP(hipMemcpyAsync(hv.data(), p.A.val, vb * nnz, hipMemcpyDeviceToHost, st));
        FH_HIP(hipStreamSynchronize(st));
        const int w = cplx_vals ? 2 : 1;
        for (long q = 0; q < nnz && S->csym; ++q)
            for (int k = 0; k < w; ++k)
                if (hv[(size_t)q * w + k] != hv[(size_t)at2a[q] * w + k]) S->csym = false;
    }
    FH_HIP(hipStreamSynchronize(st));
    ilu_chunk_defaults(*S);
}

void sparse_destroy(SparseState* s) { delete s; }

// ---------------------------------------------------------------------------
// per-node factorizations (kept across calls for the same node set)
// ---------------------------------------------------------------------------
static void ensure_factors(Ctx& c, SparseState& S, int ne, const cplx* z, bool need32, const fh_opts& o,
                           fh_report* rep) {
    hipStream_t st = c.stream;
    bool reuse = o.save_factors && (int)S.fact_z.size() == ne;
    if (reuse)
        for (int j = 0; j < ne; ++j) reuse = reuse && S.fact_z[j] == z[j];
    const int n = S.n;
    const long nnzM = S.nnzM;
    if (!reuse) {
        S.fact_z.clear();
        S.fact_prec = -1;
        zd* zd_ = (zd*)S.zdev.ensure(sizeof(zd) * ne);
        FH_HIP(hipMemcpyAsync(zd_, z, sizeof(zd) * ne, hipMemcpyHostToDevice, st));
        zd* lu = (zd*)S.lu64.ensure(sizeof(zd) * nnzM * ne);
        zd* luT = (zd*)S.luT64.ensure(sizeof(zd) * nnzM * ne);
        zd* dinv = (zd*)S.dinv64.ensure(sizeof(zd) * (size_t)n * ne);
        zd* jd = (zd*)S.jd64.ensure(sizeof(zd) * (size_t)n * ne);
        form_mvals(st, S, ne, zd_, lu);
        jacobi_diag(st, S, ne, lu, jd);      // 1/(z_j - a_ii) from the unfactored values
        ilu0_factor(st, S, ne, lu, luT, dinv);
        // level-packed values of the four sweeps
        const SweepDev* sws[4] = {&S.swL, &S.swU, &S.swUT, &S.swLT};
        const int vi[4] = {0, 1, 3, 5}, di[4] = {-1, 2, 4, -1};
        for (int q = 0; q < 4; ++q) {
            zd* ell = (zd*)S.pk64[vi[q]].ensure(sizeof(zd) * std::max<size_t>(1, (size_t)sws[q]->K * n * ne));
            zd* dg = di[q] >= 0 ? (zd*)S.pk64[di[q]].ensure(sizeof(zd) * (size_t)n * ne) : nullptr;
            pack_sweep_vals(st, *sws[q], n, ne, nnzM, lu, ell, dg);
        }
        // zero or non-finite pivots
        std::vector<zd> hdv((size_t)n * ne);
        FH_HIP(hipMemcpyAsync(hdv.data(), dinv, sizeof(zd) * hdv.size(), hipMemcpyDeviceToHost, st));
        FH_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < ne; ++j)
            for (int i = 0; i < n; ++i) {
                const zd v = hdv[(size_t)j * n + i];
                if (!std::isfinite(v.re) || !std::isfinite(v.im)) {
                    if (rep) rep->bad_node = j;
                    throw Error(FH_SINGULAR_SHIFT, "zero pivot in ILU(0) of (z_j - A) at node " + std::to_string(j));
                }
            }
        if (rep) rep->n_factor += ne;
        S.fact_z.assign(z, z + ne);
        S.fact_prec = 0;
    }
    if (need32 && S.fact_prec < 1) {
        to_single(st, nnzM * ne, (const zd*)S.lu64.p, (cf*)S.lu32.ensure(sizeof(cf) * nnzM * ne));
        to_single(st, nnzM * ne, (const zd*)S.luT64.p, (cf*)S.luT32.ensure(sizeof(cf) * nnzM * ne));
        to_single(st, (long)n * ne, (const zd*)S.dinv64.p, (cf*)S.dinv32.ensure(sizeof(cf) * (size_t)n * ne));
        to_single(st, (long)n * ne, (const zd*)S.jd64.p, (cf*)S.jd32.ensure(sizeof(cf) * (size_t)n * ne));
        for (int q = 0; q < 6; ++q) {
            if (!S.pk64[q].p) continue;
            const size_t cnt = S.pk64[q].bytes / sizeof(zd);
            to_single(st, (long)cnt, (const zd*)S.pk64[q].p, (cf*)S.pk32[q].ensure(sizeof(cf) * cnt));
        }
        S.fact_prec = 1;
    }
}

// ILU(0) factors (and the Jacobi diagonal) are needed by the preconditioner or its fallback
static bool needs_factors(const fh_opts& o) {
    const int p = o.precond == FH_PC_LEARNED ? o.fallback : o.precond;
    return p == FH_PC_ILU0 || p == FH_PC_JACOBI;
}

template <typename T>
static IluApplyArgs<T> ilu_args(SparseState& S, int m, int precond) {
    IluApplyArgs<T> a;
    const bool d = sizeof(T) == sizeof(double);
    a.n = S.n;
    a.m = m;
    a.cw = std::max(1, std::min(d ? S.ilu_cw64 : S.ilu_cw32, m));
    // wide levels (a 1,024-point grid diagonal): fewer columns per workgroup,
    // so that one level of the complex-FP32 sweep stays within 2,048 items
    if (!d) {
        const int wmax = std::max(std::max(S.swL.wmax, S.swU.wmax), std::max(S.swUT.wmax, S.swLT.wmax));
        if (wmax > 0) a.cw = std::max(1, std::min(a.cw, 2048 / wmax));
    }
    a.node_of = (const int*)S.node_of.p;
    a.side_of = (const int*)S.side_of.p;
    a.fwd[0] = S.swL;
    a.bwd[0] = S.swU;
    a.fwd[1] = S.swUT;
    a.bwd[1] = S.swLT;
    DBuf* pk = d ? S.pk64 : S.pk32;
    a.fval[0] = (const Cx<T>*)pk[0].p;
    a.fdiag[0] = nullptr;
    a.bval[0] = (const Cx<T>*)pk[1].p;
    a.bdiag[0] = (const Cx<T>*)pk[2].p;
    a.fval[1] = (const Cx<T>*)pk[3].p;
    a.fdiag[1] = (const Cx<T>*)pk[4].p;
    a.bval[1] = (const Cx<T>*)pk[5].p;
    a.bdiag[1] = nullptr;
    if (precond == FH_PC_JACOBI) a.dinv = (const Cx<T>*)(d ? S.jd64.p : S.jd32.p);
    a.junk = (Cx<T>*)S.junk.ensure(sizeof(Cx<double>) * ILU_JUNK);
    if (!d) a.blk = &S.blk;
    return a;
}

// batch: systems [0, nright) use A with shift z (side 0), [nright, nsys) use A^H with conj(z)
struct Batch {
    int nsys = 0, nright = 0, m = 0;
};

template <typename T>
static void apply_M(Ctx& c, SparseState& S, const Batch& b, const Cx<T>* shifts, T alpha, const Cx<T>* X,
                    const Cx<T>* Yadd, Cx<T>* Out) {
    const long blk = (long)S.n * b.m;
    spmm<T>(c.stream, S.A, false, S.n, b.m, b.nright, shifts, alpha, X, Yadd, Out);
    if (b.nsys > b.nright)
        spmm<T>(c.stream, S.AT, true, S.n, b.m, b.nsys - b.nright, shifts + b.nright, alpha, X + b.nright * blk,
                Yadd ? Yadd + b.nright * blk : nullptr, Out + b.nright * blk);
}

template <typename T>
static void apply_P(Ctx& c, SparseState& S, const Batch& b, int precond, Cx<T>* X, Cx<T>* Out, const T* scale) {
    if (precond == FH_PC_LEARNED) {
        // operator shift and side of every system (FP64 shifts, set by solve_batch)
        // Krylov vectors have unit columns (stopped columns are zero and unused)
        net_apply<T>(c, *S.net, b.nsys, b.m, X, (const zd*)S.shifts64.p, (const int*)S.side_of.p, Out, true);
        return;
    }
    IluApplyArgs<T> a = ilu_args<T>(S, b.m, precond);
    if (precond == FH_PC_ILU0) ilu_apply<T>(c.stream, a, b.nsys, X, Out, scale);
    else {
        if (precond == FH_PC_NONE) a.dinv = nullptr;                 // identity
        jacobi_apply<T>(c.stream, a, b.nsys, X, Out, scale);
    }
}

// Z = P^{-1} V_k and W = M Z of a Krylov step with the fixed ILU(0)
// preconditioner in complex FP32: when the sweep runs in its blocked layout
// the product reads that layout directly (Z is then not written).  False
// when the step is not of that kind (nothing done).
template <typename T>
static bool ilu_step(Ctx& c, SparseState& S, const Batch& b, int precond, bool flex, const Cx<T>* shifts,
                     Cx<T>* Vk, Cx<T>* Zk, Cx<T>* W) {
    if constexpr (sizeof(T) == 4) {
        if (flex || precond != FH_PC_ILU0) return false;
        SpmmAfter f;
        f.S = &S;
        f.nright = b.nright;
        f.shifts = shifts;
        f.alpha = 1.f;
        f.W = W;
        const IluApplyArgs<T> a = ilu_args<T>(S, b.m, precond);
        if (!ilu_apply<T>(c.stream, a, b.nsys, Vk, Zk, nullptr, &f)) apply_M<T>(c, S, b, shifts, T(1), Zk, nullptr, W);
        return true;
    } else {
        return false;
    }
}

struct SolveStats {
    long long steps = 0;
    double relres = 0.0;
    int cycles = 0;
    int fallback = 0;   // 1 if the learned preconditioner was replaced
};

// a restart cycle with the learned preconditioner must at least halve the
// worst relative residual, else the fallback preconditioner takes over
constexpr double LEARNED_STALL = 0.5;

// GMRES(restart), right preconditioned, every column of every system in lockstep.
// Solves M_s x = b_s; x starts at zero.  bn: device column norms of b (C doubles).
template <typename T>
static SolveStats gmres(Ctx& c, SparseState& S, const Batch& b, const Cx<T>* shifts, const Cx<T>* B, Cx<T>* X,
                        int restart, int max_cycles, double tol, int precond, const double* bn, int fallback,
                        int orth_passes) {
    hipStream_t st = c.stream;
    const int n = S.n, m = b.m, C = b.nsys * m, KP = restart + 1;
    const long vstride = (long)b.nsys * n * m;
    SolveStats stats;
    Cx<T>* V = (Cx<T>*)S.V.ensure(sizeof(Cx<T>) * vstride * (restart + 1));
    Cx<T>* Z = (Cx<T>*)S.Z.ensure(sizeof(Cx<T>) * vstride);
    // a nonlinear (learned) preconditioner needs the flexible variant: keep
    // every Z_k and update x with them directly
    const bool flex = (precond == FH_PC_LEARNED);
    Cx<T>* Zf = flex ? (Cx<T>*)S.Zf.ensure(sizeof(Cx<T>) * vstride * restart) : nullptr;
    zd* Hs = (zd*)S.Hs.ensure(sizeof(zd) * (size_t)restart * KP * C);
    double* cs = (double*)S.cs.ensure(sizeof(double) * (size_t)restart * C);
    zd* sn = (zd*)S.sn.ensure(sizeof(zd) * (size_t)restart * C);
    zd* g = (zd*)S.g.ensure(sizeof(zd) * (size_t)KP * C);
    double* resid = (double*)S.resid.ensure(sizeof(double) * C);
    double* vscale = (double*)S.vscale.ensure(sizeof(double) * C);
    int* kuse = (int*)S.kuse.ensure(sizeof(int) * C);
    zd* y = (zd*)S.y.ensure(sizeof(zd) * (size_t)restart * C);
    zd* h1 = (zd*)S.h1.ensure(sizeof(zd) * (size_t)KP * C);
    zd* h2 = (zd*)S.h2.ensure(sizeof(zd) * (size_t)KP * C);
    double* hnorm = (double*)S.hnorm.ensure(sizeof(double) * C);
    double* beta = (double*)S.beta.ensure(sizeof(double) * C);
    std::vector<double> hb(C), hbn(C);
    std::vector<int> hk(C);
    // delayed reorthogonalization: bases of up to 32 vectors (restart <= 31);
    // longer cycles use classical Gram-Schmidt with reorthogonalization
    const bool delayed = orth_passes == 3 && restart <= 31;
    if (orth_passes == 3 && !delayed) orth_passes = 2;
    DcgsState dstate;
    if (delayed) {
        dstate.KP = KP;
        dstate.Hs = Hs;
        dstate.sn = sn;
        dstate.g = g;
        dstate.cs = cs;
        dstate.resid = resid;
        dstate.vscale = vscale;
        dstate.kuse = kuse;
        dstate.bnorm = bn;
        dstate.Hraw = (zd*)S.Hraw.ensure(sizeof(zd) * (size_t)restart * KP * C);
        dstate.htent = (zd*)S.htent.ensure(sizeof(zd) * (size_t)KP * C);
        dstate.tau = (double*)S.tau.ensure(sizeof(double) * C);
        dstate.coef = (zd*)S.dcoef.ensure(sizeof(zd) * (size_t)2 * KP * C);
        dstate.scv = (double*)S.scv.ensure(sizeof(double) * C);
        dstate.scw = (double*)S.scw.ensure(sizeof(double) * C);
        dstate.D = (zd*)S.dots.ensure(sizeof(zd) * (size_t)(2 * 32 + 3) * C);
        dstate.part = &S.part;
    }
    FH_HIP(hipMemsetAsync(X, 0, sizeof(Cx<T>) * vstride, st));
    FH_HIP(hipMemcpyAsync(hbn.data(), bn, sizeof(double) * C, hipMemcpyDeviceToHost, st));
    double prev_worst = 0.0;
    for (int cyc = 0; cyc < max_cycles + 1; ++cyc) {
        // r = b - M x into V_0
        if (cyc == 0) FH_HIP(hipMemcpyAsync(V, B, sizeof(Cx<T>) * vstride, hipMemcpyDeviceToDevice, st));
        else apply_M<T>(c, S, b, shifts, T(-1), X, B, V);
        colnorms<T>(st, n, m, b.nsys, V, beta, S.part);
        FH_HIP(hipMemcpyAsync(hb.data(), beta, sizeof(double) * C, hipMemcpyDeviceToHost, st));
        FH_HIP(hipStreamSynchronize(st));
        double worst = 0.0;
        for (int k = 0; k < C; ++k) {
            // an overflow in the operator or the preconditioner (e.g. an
            // unstable incomplete factorization in complex FP32) must not pass
            // for convergence
            if (!std::isfinite(hb[k]))
                throw Error(FH_NONFINITE, "non-finite residual in the Krylov solve (system " +
                                              std::to_string(k / m) + "): the operator or preconditioner overflowed");
            worst = std::max(worst, hbn[k] > 0 ? hb[k] / hbn[k] : 0.0);
        }
        stats.relres = worst;
        if (!(worst > tol) || cyc == max_cycles) break;
        if (precond == FH_PC_LEARNED && cyc > 0 && !(worst < LEARNED_STALL * prev_worst)) {
            precond = fallback;            // flexible updates stay valid for any preconditioner
            stats.fallback = 1;
        }
        prev_worst = worst;
        stats.cycles++;
        gmres_start(st, C, KP, restart, beta, bn, tol, g, vscale, kuse);
        scale_inplace<T>(st, n, m, b.nsys, V, vscale);                  // V_0 = r / beta
        int kexec = 0;
        for (int k = 0; k < restart; ++k) {
            Cx<T>* Vk = V + (long)k * vstride;
            Cx<T>* Vk1 = V + (long)(k + 1) * vstride;
            Cx<T>* Zk = flex ? Zf + (long)k * vstride : Z;
            if (!ilu_step<T>(c, S, b, precond, flex, shifts, Vk, Zk, Vk1)) {
                apply_P<T>(c, S, b, precond, Vk, Zk, (const T*)nullptr);    // Z = P^{-1} V_k
                apply_M<T>(c, S, b, shifts, T(1), Zk, nullptr, Vk1);        // W = M Z
            }
            kexec = k + 1;
            stats.steps++;
            if (delayed) {
                // V_k reorthogonalized, W -> tentative V_{k+1}, column k - 1 final
                dcgs_step<T>(st, n, m, b.nsys, k, V, vstride, Vk1, dstate, flex ? 1 : 0, 0, tol);
            } else {
                cgs2<T>(st, n, m, b.nsys, k + 1, V, vstride, Vk1, h1, h2, hnorm, S.part, orth_passes);
                givens_step(st, C, k, KP, h1, h2, hnorm, Hs, cs, sn, g, resid, vscale, kuse, bn, tol);
                scale_inplace<T>(st, n, m, b.nsys, Vk1, vscale);        // V_{k+1} = W / h_{k+1,k}
            }
            FH_HIP(hipMemcpyAsync(hk.data(), kuse, sizeof(int) * C, hipMemcpyDeviceToHost, st));
            FH_HIP(hipStreamSynchronize(st));
            // delayed: the columns known to have stopped are those of column k - 1
            const int need = delayed ? k : k + 1;
            bool any = false;
            for (int q = 0; q < C && !any; ++q) any = hk[q] > need;
            if (!any) break;
        }
        if (delayed) {
            // the last column is still tentative: finalize it (dots of the
            // tentative V_kexec only) where a column still runs
            bool any = false;
            for (int q = 0; q < C && !any; ++q) any = hk[q] >= kexec;
            if (any) dcgs_step<T>(st, n, m, b.nsys, kexec, V, vstride, (Cx<T>*)nullptr, dstate, flex ? 1 : 0, 1, tol);
        }
        if (flex) {
            // x += Z y
            gmres_update_prep<T>(st, n, m, b.nsys, kexec, KP, Hs, g, kuse, y, Zf, vstride, Z);
            add_same<T>(st, vstride, Z, X);
        } else {
            // x += P^{-1} (V y)
            gmres_update_prep<T>(st, n, m, b.nsys, kexec, KP, Hs, g, kuse, y, V, vstride, Z);
            Cx<T>* tmp = V + (long)kexec * vstride;   // free after the cycle
            apply_P<T>(c, S, b, precond, Z, tmp, (const T*)nullptr);
            add_same<T>(st, vstride, tmp, X);                           // x += P^{-1} V y
        }
    }
    return stats;
}

// operator shifts per system: z for a right system, conj(z) for a left one
template <typename T>
static Cx<T>* upload_op_shifts(Ctx& c, SparseState& S, int nsys, const cplx* zsys, const int* side) {
    std::vector<Cx<T>> h(nsys);
    for (int s = 0; s < nsys; ++s) h[s] = Cx<T>{T(zsys[s].real()), T(side[s] ? -zsys[s].imag() : zsys[s].imag())};
    DBuf& d = sizeof(T) == sizeof(double) ? S.shifts64 : S.shifts32;
    Cx<T>* p = (Cx<T>*)d.ensure(sizeof(Cx<T>) * nsys);
    FH_HIP(hipMemcpyAsync(p, h.data(), sizeof(Cx<T>) * nsys, hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
    return p;
}

// Solve the nsys shifted systems of a batch: system s uses the factors of node
// node_of[s] with node value zsys[s]; sides: the first nright systems are
// right systems (z - A) x = b, the others left systems (z - A)^H x = b.
// B64, X64: [nsys][n][m] FP64.
static SolveStats solve_batch(Ctx& c, SparseState& S, int nsys, int nright, const int* node_of, const cplx* zsys, int m,
                              const zd* B64, zd* X64, const fh_opts& o) {
    hipStream_t st = c.stream;
    Batch b;
    b.nsys = nsys;
    b.nright = nright;
    b.m = m;
    const int n = S.n, C = b.nsys * m;
    const long len = (long)b.nsys * n * m;
    std::vector<int> side_of(b.nsys);
    for (int s = 0; s < b.nsys; ++s) side_of[s] = s >= nright;
    FH_HIP(hipMemcpyAsync(S.node_of.ensure(sizeof(int) * b.nsys), node_of, sizeof(int) * b.nsys,
                          hipMemcpyHostToDevice, st));
    FH_HIP(hipMemcpyAsync(S.side_of.ensure(sizeof(int) * b.nsys), side_of.data(), sizeof(int) * b.nsys,
                          hipMemcpyHostToDevice, st));
    const int precond = o.precond;
    FH_REQUIRE(precond != FH_PC_LEARNED || S.net, -1, "learned preconditioner requested but no network is attached");
    double* bn = (double*)S.bn64.ensure(sizeof(double) * C);
    colnorms<double>(st, n, m, b.nsys, B64, bn, S.part);
    const int restart = std::max(1, o.restart);
    zd* sh64 = upload_op_shifts<double>(c, S, nsys, zsys, side_of.data());
    if (o.precision == FH_PREC_FP64) {
        // buffers of the mixed path only: give their memory back for the
        // (twice as large) FP64 Krylov basis
        S.bufR.release();
        S.b32.release();
        S.x32.release();
        S.blk.release();
        if (precond != FH_PC_LEARNED) S.Zf.release();
        return gmres<double>(c, S, b, sh64, B64, X64, restart, std::max(1, o.max_restarts), o.inner_tol, precond, bn,
                             o.fallback, o.orth == 1 ? 1 : (o.orth == 2 ? 3 : 2));
    }
    // complex FP32 inner solves wrapped in FP64 iterative refinement
    cf* sh32 = upload_op_shifts<float>(c, S, nsys, zsys, side_of.data());
    zd* R = (zd*)S.bufR.ensure(sizeof(zd) * len);
    cf* b32 = (cf*)S.b32.ensure(sizeof(cf) * len);
    cf* x32 = (cf*)S.x32.ensure(sizeof(cf) * len);
    double* rn = (double*)S.rn64.ensure(sizeof(double) * C);
    double* sc = (double*)S.sc64.ensure(sizeof(double) * C);
    std::vector<double> hrn(C), hbn(C), hsc(C);
    FH_HIP(hipMemcpyAsync(hbn.data(), bn, sizeof(double) * C, hipMemcpyDeviceToHost, st));
    FH_HIP(hipMemsetAsync(X64, 0, sizeof(zd) * len, st));
    FH_HIP(hipMemcpyAsync(R, B64, sizeof(zd) * len, hipMemcpyDeviceToDevice, st));
    SolveStats tot;
    int pc = precond;
    for (int it = 0; it <= std::max(1, o.max_refine); ++it) {
        colnorms<double>(st, n, m, b.nsys, R, rn, S.part);
        FH_HIP(hipMemcpyAsync(hrn.data(), rn, sizeof(double) * C, hipMemcpyDeviceToHost, st));
        FH_HIP(hipStreamSynchronize(st));
        double worst = 0.0;
        for (int k = 0; k < C; ++k) worst = std::max(worst, hbn[k] > 0 ? hrn[k] / hbn[k] : 0.0);
        tot.relres = worst;
        if (!(worst > o.inner_tol) || it == std::max(1, o.max_refine)) break;
        for (int k = 0; k < C; ++k) hsc[k] = hrn[k] > 0 ? 1.0 / hrn[k] : 0.0;
        FH_HIP(hipMemcpyAsync(sc, hsc.data(), sizeof(double) * C, hipMemcpyHostToDevice, st));
        scale_cols_cast<float>(st, n, m, b.nsys, R, sc, b32);          // unit columns in FP32
        double* ones = (double*)S.bn32.ensure(sizeof(double) * C);     // |b32 columns| = 1 (or 0)
        colnorms<float>(st, n, m, b.nsys, b32, ones, S.part);
        SolveStats s32 = gmres<float>(c, S, b, sh32, b32, x32, restart, std::max(1, o.max_restarts),
                                      o.mixed_inner_tol, pc, ones, o.fallback, o.orth == 1 ? 1 : (o.orth == 2 ? 3 : 2));
        tot.steps += s32.steps;
        tot.fallback |= s32.fallback;
        if (s32.fallback) pc = o.fallback;     // later refinement steps keep the fallback
        tot.cycles += s32.cycles;
        FH_HIP(hipMemcpyAsync(sc, hrn.data(), sizeof(double) * C, hipMemcpyHostToDevice, st));
        axpy_cols<float>(st, n, m, b.nsys, x32, sc, X64);               // x += |r| d
        apply_M<double>(c, S, b, sh64, -1.0, X64, B64, R);               // r = b - M x in FP64
    }
    return tot;
}

// all 2 ne systems of the filter: right systems of nodes 0..ne-1, then left ones
static SolveStats solve_all(Ctx& c, SparseState& S, int ne, const cplx* z, int m, const zd* B64, zd* X64,
                            const fh_opts& o) {
    std::vector<int> node_of(2 * ne);
    std::vector<cplx> zsys(2 * ne);
    for (int s = 0; s < 2 * ne; ++s) { node_of[s] = s % ne; zsys[s] = z[s % ne]; }
    return solve_batch(c, S, 2 * ne, ne, node_of.data(), zsys.data(), m, B64, X64, o);
}

// public: solve (z_s - A) X_s = B_s (right) / (z_s - A)^H X_s = B_s (left) for a
// batch whose right systems come first; one ILU(0) per system (cached)
void sparse_shifted_solve(Ctx& c, Prob& p, int nsys, const cplx* z, const int* sides, int m, const zd* B, zd* X,
                          const fh_opts& o, fh_report* rep) {
    SparseState& S = *p.sp;
    int nright = 0;
    while (nright < nsys && sides[nright] == 0) ++nright;
    if (needs_factors(o)) ensure_factors(c, S, nsys, z, o.precision == FH_PREC_MIXED, o, rep);
    std::vector<int> node_of(nsys);
    for (int s = 0; s < nsys; ++s) node_of[s] = s;
    SolveStats st = solve_batch(c, S, nsys, nright, node_of.data(), z, m, B, X, o);
    FH_HIP(hipStreamSynchronize(c.stream));
    if (rep) {
        rep->n_fallback += st.fallback ? nsys : 0;
        rep->n_solve += nsys;
        rep->inner_steps = st.steps;
        rep->inner_relres = st.relres;
    }
}

// ---------------------------------------------------------------------------
// contour filter on a CSR problem (B = I)
// ---------------------------------------------------------------------------
// Nodes per batch of the sparse filter: opts.batch_nodes, or as many as fit in
// 65 % of the device memory with the workspace of one system (right or left)
// estimated as its Krylov basis, flexible directions, work copies and the
// filter's right-hand side and solution blocks (the rest holds the FEAST
// iteration's n x m0 blocks, the factors and the caller's arrays: about
// 40 GB for the 1,048,576-point workload with m0 = 160).
static int filter_chunk(const SparseState& S, int ne, int m, const fh_opts& o) {
    if (o.batch_nodes > 0) return std::min(ne, o.batch_nodes);
    const double elems = (double)S.n * m;
    const int restart = std::max(1, o.restart);
    const bool flex = o.precond == FH_PC_LEARNED;
    const double b = o.precision == FH_PREC_MIXED ? 8.0 : 16.0;       // bytes of a Krylov entry
    double per_sys = elems * (b * (restart + 2 + (flex ? restart : 0)) + 2 * 16.0);
    // FP64 residual, FP32 rhs / solution, blocked-layout copy of the ILU(0) sweep
    if (o.precision == FH_PREC_MIXED) per_sys += elems * (16.0 + 3 * 8.0);
    size_t freeb = 0, total = 0;
    FH_HIP(hipMemGetInfo(&freeb, &total));
    const double budget = 0.65 * (double)total;
    const int g = (int)std::floor(budget / ((o.sym ? 1.0 : 2.0) * per_sys));
    return std::max(1, std::min(ne, g));
}

// Nodes symmetric about the real axis: each node off the axis has a partner
// z_k = conj(z_j) with w_k = conj(w_j).  fz: the upper and real-axis nodes;
// fmap[j]: index in fz of node j (a lower node: of its partner); flip[j] = 1
// for a lower node.  False (and fmap the identity) when some node has no
// partner.
static bool pair_nodes(int ne, const cplx* z, const cplx* w, std::vector<int>& fmap, std::vector<int>& flip,
                       std::vector<cplx>& fz) {
    fmap.resize(ne);
    flip.assign(ne, 0);
    fz.clear();
    for (int j = 0; j < ne; ++j) fmap[j] = j;
    std::vector<int> partner(ne, -1);
    for (int j = 0; j < ne; ++j) {
        if (z[j].imag() == 0.0) continue;
        for (int k = 0; k < ne; ++k) {
            const double tz = 1e-13 * (1.0 + std::abs(z[j])), tw = 1e-13 * (1.0 + std::abs(w[j]));
            if (k != j && std::abs(z[k] - std::conj(z[j])) <= tz && std::abs(w[k] - std::conj(w[j])) <= tw) {
                partner[j] = k;
                break;
            }
        }
        if (partner[j] < 0) return false;
    }
    std::vector<int> fidx(ne, -1);
    for (int j = 0; j < ne; ++j)
        if (z[j].imag() >= 0.0) { fidx[j] = (int)fz.size(); fz.push_back(z[j]); }
    for (int j = 0; j < ne; ++j) {
        if (z[j].imag() >= 0.0) fmap[j] = fidx[j];
        else { fmap[j] = fidx[partner[j]]; flip[j] = 1; }
    }
    return true;
}

bool sparse_conj_closed(const Prob& p, int ne, const cplx* z, const cplx* w, const fh_opts& o) {
    if (p.dense || o.conj_pairs != 2 || p.sp->A.complex_vals) return false;
    std::vector<int> fmap, flip;
    std::vector<cplx> fz;
    return pair_nodes(ne, z, w, fmap, flip, fz);
}

void sparse_filter(Ctx& c, Prob& p, int ne, const cplx* z, const cplx* w, int m, const zd* Y, const zd* Yh, zd* Q,
                   zd* Qh, const fh_opts& o, fh_report* rep, const cplx* lam, const int* cpart) {
    FH_REQUIRE(m >= 1 && m <= 256, -6, "sparse filter: m0 must be in [1, 256]");
    SparseState& S = *p.sp;
    // complex symmetric problems: the left subspace is the conjugate of the
    // right one (section on reduced workloads, complex symmetric case), so
    // only the right systems are solved
    const bool sym = o.sym == 1;
    FH_REQUIRE(!sym || S.csym, -2, "opts.sym = 1 needs a complex symmetric matrix (A = A^T)");
    // right systems only: complex symmetric problems, and callers without a
    // left block (the eigenvalue-count estimate)
    const bool right_only = sym || Yh == nullptr;
    hipStream_t st = c.stream;
    const int n = S.n;
    const long blk = (long)n * m;
    // Real A and a node set symmetric about the real axis (each lower node the
    // conjugate of an upper one, with the conjugate weight): for real A,
    // (conj(z) - A)^{-1} b = conj((z - A)^{-1} conj(b)) and
    // (conj(z) - A)^{-H} b = conj((z - A)^{-H} conj(b)), and the ILU(0) of
    // conj(z) - A is the conjugate of that of z - A, so only the upper (and
    // real-axis) nodes are factorized: a lower node's systems are solved as
    // its upper partner's with conjugated right-hand sides, and their
    // solutions conjugated back (the paper's real non-symmetric case with a
    // contour symmetric about the real axis: n_e/2 factorizations).
    std::vector<int> fmap, flip;
    std::vector<cplx> fz;
    const bool paired = o.conj_pairs && !S.A.complex_vals && pair_nodes(ne, z, w, fmap, flip, fz);
    if (!paired) {
        fz.assign(z, z + ne);
        fmap.resize(ne);
        flip.assign(ne, 0);
        for (int j = 0; j < ne; ++j) fmap[j] = j;
    }
    const int nf = (int)fz.size();
    // Conjugation-closed right-hand sides (conj_pairs = 2): when column
    // cp[i] of the right-hand side block is the conjugate of column i, the
    // conjugated right-hand sides a lower node needs are columns of the block
    // itself, so conj((z - A)^{-1} conj(r_i)) = conj(E[:, cp[i]]) with E the
    // upper node's solution: only the upper nodes' systems are solved, n_e/2
    // per side (Table tab:solve, real non-symmetric with a contour symmetric
    // about the real axis: n_e/2 factorizations and n_e solves).  The FEAST
    // driver passes cp for its symmetrized Ritz vectors; a direct call with
    // real Y and Yh (no Ritz values) uses cp = identity.
    std::vector<int> cp;
    if (paired && o.conj_pairs == 2) {
        if (cpart) {
            cp.assign(cpart, cpart + m);
            for (int i = 0; i < m; ++i)
                FH_REQUIRE(cp[i] >= 0 && cp[i] < m && cp[cp[i]] == i, -3, "column partners must be an involution");
        } else if (!lam) {
            int* fl = (int*)S.flag.ensure(sizeof(int));
            FH_HIP(hipMemsetAsync(fl, 0, sizeof(int), st));
            any_imag(st, blk, Y, fl);
            if (!right_only) any_imag(st, blk, Yh, fl);
            int h = 1;
            FH_HIP(hipMemcpyAsync(&h, fl, sizeof(int), hipMemcpyDeviceToHost, st));
            FH_HIP(hipStreamSynchronize(st));
            if (h == 0) {
                cp.resize(m);
                for (int i = 0; i < m; ++i) cp[i] = i;
            }
        }
    }
    const bool half = !cp.empty();
    if (needs_factors(o)) ensure_factors(c, S, nf, fz.data(), o.precision == FH_PREC_MIXED, o, rep);
    const int nnode = half ? nf : ne;      // nodes whose systems are solved
    const int g = filter_chunk(S, nnode, m, o);
    zd* Bb = (zd*)S.bufB.ensure(sizeof(zd) * blk * 2 * g);
    zd* Xb = (zd*)S.bufX.ensure(sizeof(zd) * blk * 2 * g);
    zd* T = (zd*)S.bufT.ensure(sizeof(zd) * blk * 2);
    zd* lamd = nullptr;
    // coef[side][j][i]: weight of column i of E_j (right: w_j or w_j / (z_j - lam_i); left: conjugates)
    std::vector<cplx> coef(2 * (size_t)ne * m), rho(2 * (size_t)m);
    if (lam) {
        zd* ld = (zd*)S.rho.ensure(sizeof(zd) * 3 * m);
        lamd = ld + 2 * m;
        FH_HIP(hipMemcpyAsync(lamd, lam, sizeof(zd) * m, hipMemcpyHostToDevice, st));
        ritz_residual(st, S.A, false, n, m, lamd, false, Y, T);           // R  = A Y - Y Lambda
        if (!right_only) ritz_residual(st, S.AT, true, n, m, lamd, true, Yh, T + blk);   // Rh = A^H Yh - Yh Lambda^*
        for (int i = 0; i < m; ++i) {
            cplx r = 0.0;
            for (int j = 0; j < ne; ++j) {
                const cplx cj = w[j] / (z[j] - lam[i]);
                coef[(size_t)j * m + i] = cj;
                coef[(size_t)ne * m + (size_t)j * m + i] = std::conj(cj);
                r += cj;
            }
            rho[i] = r;
            rho[m + i] = std::conj(r);
        }
    } else {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < ne; ++j) {
                coef[(size_t)j * m + i] = w[j];
                coef[(size_t)ne * m + (size_t)j * m + i] = std::conj(w[j]);
            }
    }
    zd* cd = (zd*)S.coef.ensure(sizeof(zd) * coef.size());
    zd *cu = nullptr, *cl = nullptr;
    int* cpd = nullptr;
    if (half) {
        // cu[side][f][i] / cl[side][f][i]: weights of upper node f and of its
        // lower partner (zero for a real-axis node)
        std::vector<cplx> cuh(2 * (size_t)nf * m, 0.0), clh(2 * (size_t)nf * m, 0.0);
        for (int sd = 0; sd < 2; ++sd)
            for (int j = 0; j < ne; ++j) {
                std::vector<cplx>& dst = flip[j] ? clh : cuh;
                for (int i = 0; i < m; ++i)
                    dst[(size_t)sd * nf * m + (size_t)fmap[j] * m + i] = coef[(size_t)sd * ne * m + (size_t)j * m + i];
            }
        zd* cpb = (zd*)S.coefp.ensure(sizeof(zd) * 4 * (size_t)nf * m);
        cu = cpb;
        cl = cpb + 2 * (size_t)nf * m;
        FH_HIP(hipMemcpyAsync(cu, cuh.data(), sizeof(zd) * cuh.size(), hipMemcpyHostToDevice, st));
        FH_HIP(hipMemcpyAsync(cl, clh.data(), sizeof(zd) * clh.size(), hipMemcpyHostToDevice, st));
        cpd = (int*)S.cpd.ensure(sizeof(int) * m);
        FH_HIP(hipMemcpyAsync(cpd, cp.data(), sizeof(int) * m, hipMemcpyHostToDevice, st));
    } else {
        FH_HIP(hipMemcpyAsync(cd, coef.data(), sizeof(zd) * coef.size(), hipMemcpyHostToDevice, st));
    }
    zd* rd = nullptr;
    if (lam) {
        rd = (zd*)S.rho.p;
        FH_HIP(hipMemcpyAsync(rd, rho.data(), sizeof(zd) * 2 * m, hipMemcpyHostToDevice, st));
    }
    const zd* Rr = lam ? T : Y;            // right-hand sides: residuals (or Y), replicated per node
    const zd* Rl = lam ? T + blk : Yh;
    SolveStats s;
    // nodes [j0, j1) at a time (of fz when half, else of z): their right and
    // left systems in one batch
    const int sides = right_only ? 1 : 2;
    for (int j0 = 0; j0 < nnode; j0 += g) {
        const int j1 = std::min(nnode, j0 + g), gc = j1 - j0;
        replicate<double>(st, blk, Rr, Bb, gc);
        if (!right_only) replicate<double>(st, blk, Rl, Bb + gc * blk, gc);
        std::vector<int> node_of(sides * gc);
        std::vector<cplx> zsys(sides * gc);
        for (int q = 0; q < sides * gc; ++q) {
            const int j = j0 + q % gc;
            node_of[q] = half ? j : fmap[j];
            zsys[q] = half ? fz[j] : paired ? fz[fmap[j]] : z[j];
            if (!half && flip[j]) conj_copy(st, blk, Bb + (long)q * blk, Bb + (long)q * blk);   // conj(b)
        }
        const SolveStats sc = solve_batch(c, S, sides * gc, gc, node_of.data(), zsys.data(), m, Bb, Xb, o);
        if (!half)
            for (int q = 0; q < sides * gc; ++q)
                if (flip[j0 + q % gc]) conj_copy(st, blk, Xb + (long)q * blk, Xb + (long)q * blk);
        s.steps += sc.steps;
        s.cycles += sc.cycles;
        s.relres = std::max(s.relres, sc.relres);
        s.fallback |= sc.fallback;
        const bool first = j0 == 0;
        const zd* Yr = (lam && first) ? Y : nullptr;
        const zd* Yl = (lam && first) ? Yh : nullptr;
        const zd* rr = first ? rd : nullptr;
        const zd* rl = (first && rd) ? rd + m : nullptr;
        if (half) {
            const size_t ls = (size_t)nf * m;
            filter_accum_pair(st, gc, n, m, Xb, cu + (size_t)j0 * m, cl + (size_t)j0 * m, cpd, Yr, rr, Q, !first);
            if (!right_only)
                filter_accum_pair(st, gc, n, m, Xb + gc * blk, cu + ls + (size_t)j0 * m, cl + ls + (size_t)j0 * m, cpd,
                                  Yl, rl, Qh, !first);
        } else {
            filter_accum(st, gc, n, m, Xb, cd + (size_t)j0 * m, Yr, rr, Q, !first);
            if (!right_only) filter_accum(st, gc, n, m, Xb + gc * blk, cd + (size_t)(ne + j0) * m, Yl, rl, Qh, !first);
        }
    }
    // complex symmetric: the left block is taken as conj(Y) D with
    // D = diag(conj(1 / (y_c^T y_c))), the scaling with yh_c^H y_c = 1 that
    // FEAST's left Ritz vectors have; its filter is conj(Q) D
    if (sym && Qh) conj_copy_bilin(st, n, m, Y, Q, Qh, c.partial2);
    FH_HIP(hipStreamSynchronize(st));
    if (rep) {
        rep->n_fallback += s.fallback ? sides * nnode : 0;
        rep->n_solve += sides * nnode;
        rep->inner_steps = s.steps;
        rep->inner_relres = s.relres;
    }
}

void sparse_set_net(Prob& p, NetState* net) { p.sp->net = net; }

void sparse_apply_A(Ctx& c, Prob& p, int side, int m, const zd* X, zd* Out) {
    SparseState& S = *p.sp;
    spmm<double>(c.stream, side ? S.AT : S.A, side == 1, S.n, m, 1, nullptr, -1.0, X, nullptr, Out);
}

void sparse_shifted_apply(Ctx& c, Prob& p, int side, int nsys, const cplx* shifts, int m, const zd* X, zd* Out) {
    SparseState& S = *p.sp;
    std::vector<zd> h(nsys);
    for (int s = 0; s < nsys; ++s) h[s] = zd{shifts[s].real(), shifts[s].imag()};
    zd* d = (zd*)S.shifts64.ensure(sizeof(zd) * nsys);
    FH_HIP(hipMemcpyAsync(d, h.data(), sizeof(zd) * nsys, hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
    spmm<double>(c.stream, side ? S.AT : S.A, side == 1, S.n, m, nsys, d, 1.0, X, nullptr, Out);
}

void sparse_residual_pair(Ctx& c, Prob& p, int side, int nsys, const cplx* shifts, int m, const zd* B, const zd* X,
                          const zd* Xt, zd* R, zd* E) {
    SparseState& S = *p.sp;
    std::vector<zd> h(nsys);
    for (int s = 0; s < nsys; ++s) h[s] = zd{shifts[s].real(), shifts[s].imag()};
    zd* d = (zd*)S.shifts64.ensure(sizeof(zd) * nsys);
    FH_HIP(hipMemcpyAsync(d, h.data(), sizeof(zd) * nsys, hipMemcpyHostToDevice, c.stream));
    // R = -(shift X - op(A) X) + B
    spmm<double>(c.stream, side ? S.AT : S.A, side == 1, S.n, m, nsys, d, -1.0, X, B, R);
    sub(c.stream, (long)nsys * S.n * m, Xt, X, E);
    FH_HIP(hipStreamSynchronize(c.stream));
}

void sparse_ilu0(Ctx& c, Prob& p, cplx z, zd* lu_out) {
    SparseState& S = *p.sp;
    fh_opts o;
    std::memset(&o, 0, sizeof(o));
    o.save_factors = 0;
    ensure_factors(c, S, 1, &z, false, o, nullptr);
    // values on the M pattern -> A pattern positions (plus diagonal if A has it)
    std::vector<int> a2m(S.nnzA);
    FH_HIP(hipMemcpyAsync(a2m.data(), S.a2m, sizeof(int) * S.nnzA, hipMemcpyDeviceToHost, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
    DBuf ib;
    int* idx = (int*)ib.ensure(sizeof(int) * S.nnzA);
    FH_HIP(hipMemcpyAsync(idx, a2m.data(), sizeof(int) * S.nnzA, hipMemcpyHostToDevice, c.stream));
    gather_vals(c.stream, S.nnzA, true, S.lu64.p, idx, lu_out);
    FH_HIP(hipStreamSynchronize(c.stream));
    S.fact_z.clear();   // single-node factors are not a filter node set
}

void sparse_ilu0_apply32(Ctx& c, Prob& p, cplx z, int side, int m, const cf* X, cf* Out) {
    SparseState& S = *p.sp;
    fh_opts o;
    std::memset(&o, 0, sizeof(o));
    o.save_factors = 0;
    ensure_factors(c, S, 1, &z, true, o, nullptr);
    int node = 0;
    FH_HIP(hipMemcpyAsync(S.node_of.ensure(sizeof(int)), &node, sizeof(int), hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipMemcpyAsync(S.side_of.ensure(sizeof(int)), &side, sizeof(int), hipMemcpyHostToDevice, c.stream));
    Batch b;
    b.nsys = 1;
    b.nright = side == 0 ? 1 : 0;
    b.m = m;
    DBuf xb;
    cf* xc = (cf*)xb.ensure(sizeof(cf) * (size_t)S.n * m);
    FH_HIP(hipMemcpyAsync(xc, X, sizeof(cf) * (size_t)S.n * m, hipMemcpyDeviceToDevice, c.stream));
    apply_P<float>(c, S, b, FH_PC_ILU0, xc, Out, nullptr);
    FH_HIP(hipStreamSynchronize(c.stream));
    S.fact_z.clear();
}

void sparse_ilu0_apply(Ctx& c, Prob& p, cplx z, int side, int m, const zd* X, zd* Out) {
    SparseState& S = *p.sp;
    fh_opts o;
    std::memset(&o, 0, sizeof(o));
    o.save_factors = 0;
    ensure_factors(c, S, 1, &z, false, o, nullptr);
    int node = 0;
    FH_HIP(hipMemcpyAsync(S.node_of.ensure(sizeof(int)), &node, sizeof(int), hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipMemcpyAsync(S.side_of.ensure(sizeof(int)), &side, sizeof(int), hipMemcpyHostToDevice, c.stream));
    Batch b;
    b.nsys = 1;
    b.nright = side == 0 ? 1 : 0;
    b.m = m;
    DBuf xb;
    zd* xc = (zd*)xb.ensure(sizeof(zd) * (size_t)S.n * m);
    FH_HIP(hipMemcpyAsync(xc, X, sizeof(zd) * (size_t)S.n * m, hipMemcpyDeviceToDevice, c.stream));
    apply_P<double>(c, S, b, FH_PC_ILU0, xc, Out, nullptr);
    FH_HIP(hipStreamSynchronize(c.stream));
    S.fact_z.clear();
}

}  // namespace fh
