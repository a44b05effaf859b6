// FEAST driver: contour nodes, dense contour filter, and the non-Hermitian
// FEAST iteration of the paper's complete algorithm figure (steps 0-5).
// Every step runs in this library's kernels on the handle's stream; the host
// only takes the O(m0) scalar decisions (spurious count, resize, inside test,
// convergence) from values copied back once per step.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <cstdio>
#include <cstdlib>

#include "fh_dgroup.h"
#include "fh_internal.h"

namespace fh {

static const double PI = 3.14159265358979323846;

// Trapezoidal rule on z(t) = c + e^{i phi}(a cos t + i b sin t), t_j = 2 pi (j - 1/2)/ne,
// w_j = z'(t_j)/(i ne)  (Sections 1 and 2.1; eq:rational)
static void polygon_nodes(const fh_contour& ct, std::vector<cplx>& z, std::vector<cplx>& w);

void contour_nodes(const fh_contour& ct, std::vector<cplx>& z, std::vector<cplx>& w) {
    if (ct.nv >= 3) {
        polygon_nodes(ct, z, w);
        return;
    }
    const int ne = ct.ne;
    z.resize(ne);
    w.resize(ne);
    const cplx c(ct.c_re, ct.c_im), rot = std::polar(1.0, ct.angle);
    const double a = ct.a, b = ct.ratio * ct.a;
    for (int j = 0; j < ne; ++j) {
        const double t = 2.0 * PI * (j + 0.5) / ne;
        z[j] = c + rot * cplx(a * std::cos(t), b * std::sin(t));
        const cplx dz = rot * cplx(-a * std::sin(t), b * std::cos(t));
        w[j] = dz / (cplx(0.0, 1.0) * double(ne));
    }
}

// polygon: composite trapezoid rule on each side (ne / nv intervals), nodes
// at the interval ends; the weight of a node is (h_prev + h_next) / (2 * 2 pi i)
// with h the complex interval steps beside it, counterclockwise orientation
static void polygon_nodes(const fh_contour& ct, std::vector<cplx>& z, std::vector<cplx>& w) {
    const int nv = ct.nv, per = ct.ne / nv;
    std::vector<cplx> v(nv);
    double area2 = 0.0;
    for (int k = 0; k < nv; ++k) v[k] = cplx(ct.verts[2 * k], ct.verts[2 * k + 1]);
    for (int k = 0; k < nv; ++k) {
        const cplx a = v[k], b = v[(k + 1) % nv];
        area2 += a.real() * b.imag() - b.real() * a.imag();
    }
    if (area2 < 0.0) std::reverse(v.begin(), v.end());
    const cplx twopii(0.0, 2.0 * PI);
    z.clear();
    w.clear();
    for (int k = 0; k < nv; ++k) {
        const cplx h = (v[(k + 1) % nv] - v[k]) / double(per);
        const cplx hp = (v[k] - v[(k + nv - 1) % nv]) / double(per);
        for (int q = 0; q < per; ++q) {
            z.push_back(v[k] + double(q) * h);
            w.push_back((q == 0 ? 0.5 * (hp + h) : h) / twopii);
        }
    }
}

static cplx polygon_centroid(const fh_contour& ct) {
    cplx g = 0.0;
    for (int k = 0; k < ct.nv; ++k) g += cplx(ct.verts[2 * k], ct.verts[2 * k + 1]);
    return g / double(ct.nv);
}

double contour_alpha(const fh_contour& ct) {
    if (ct.nv >= 3) {
        const cplx g = polygon_centroid(ct);
        double r = 0.0;
        for (int k = 0; k < ct.nv; ++k) r = std::max(r, std::abs(cplx(ct.verts[2 * k], ct.verts[2 * k + 1]) - g));
        return std::abs(g) + r;
    }
    return std::abs(cplx(ct.c_re, ct.c_im)) + std::max(ct.a, ct.ratio * ct.a);
}

static bool inside_contour(const fh_contour& ct, cplx lam) {
    if (!std::isfinite(lam.real()) || !std::isfinite(lam.imag())) return false;
    if (ct.nv >= 3) {                                 // even-odd ray casting along +Re
        bool in = false;
        for (int k = 0, l = ct.nv - 1; k < ct.nv; l = k++) {
            const double xk = ct.verts[2 * k], yk = ct.verts[2 * k + 1];
            const double xl = ct.verts[2 * l], yl = ct.verts[2 * l + 1];
            if ((yk > lam.imag()) != (yl > lam.imag()) &&
                lam.real() < xk + (lam.imag() - yk) * (xl - xk) / (yl - yk))
                in = !in;
        }
        return in;
    }
    const cplx u = (lam - cplx(ct.c_re, ct.c_im)) * std::polar(1.0, -ct.angle);
    const double a = ct.a, b = ct.ratio * ct.a;
    const double q = (u.real() / a) * (u.real() / a) + (u.imag() / b) * (u.imag() / b);
    return q < 1.0;
}

static cplx rational(int ne, const cplx* z, const cplx* w, cplx lam) {
    cplx s = 0.0;
    for (int j = 0; j < ne; ++j) s += w[j] / (z[j] - lam);
    return s;
}

static void sync(Ctx& c) { FH_HIP(hipStreamSynchronize(c.stream)); }

// Column partners of Ritz values that come in conjugate pairs (a real pencil
// whose search subspace is closed under conjugation): i and k are partners
// when each is the other's nearest conjugate (k = i for a real value); the
// columns left over are paired greedily, each with the nearest conjugate
// among them, so the result is always an involution.  Non-finite values stay
// alone.
static std::vector<int> conj_partners(const cplx* lam, int m) {
    auto fin = [&](int i) { return std::isfinite(lam[i].real()) && std::isfinite(lam[i].imag()); };
    std::vector<int> cp(m, -1), near(m);
    for (int i = 0; i < m; ++i) {
        near[i] = i;
        if (!fin(i)) continue;
        double bd = std::abs(lam[i] - std::conj(lam[i]));
        for (int k = 0; k < m; ++k)
            if (k != i && fin(k)) {
                const double d = std::abs(lam[k] - std::conj(lam[i]));
                if (d < bd) { bd = d; near[i] = k; }
            }
    }
    for (int i = 0; i < m; ++i)
        if (near[near[i]] == i) cp[i] = near[i];
    for (int i = 0; i < m; ++i) {
        if (cp[i] >= 0) continue;
        int best = i;
        double bd = fin(i) ? std::abs(lam[i] - std::conj(lam[i])) : 0.0;
        if (fin(i))
            for (int k = i + 1; k < m; ++k)
                if (cp[k] < 0 && fin(k)) {
                    const double d = std::abs(lam[k] - std::conj(lam[i]));
                    if (d < bd) { bd = d; best = k; }
                }
        cp[i] = best;
        cp[best] = i;
    }
    return cp;
}

// FH_VERBOSE=1 prints one line per FEAST iteration to stderr
static int verbose() {
    static const int v = [] {
        const char* e = std::getenv("FH_VERBOSE");
        return e ? std::atoi(e) : 0;
    }();
    return v;
}

template <typename T>
static void to_host(Ctx& c, T* dst, const void* src, size_t count) {
    FH_HIP(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyDeviceToHost, c.stream));
    sync(c);
}
// small uploads; synchronous so that the host source may go out of scope
template <typename T>
static void to_dev(Ctx& c, void* dst, const T* src, size_t count) {
    FH_HIP(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, c.stream));
    sync(c);
}

// ---------------------------------------------------------------------------
// operators
// ---------------------------------------------------------------------------
void apply_A(Ctx& c, Prob& p, int side, int m, const zd* X, zd* Out) {
    if (!p.dense) { sparse_apply_A(c, p, side, m, X, Out); return; }
    const zd* A = (const zd*)p.A.val;
    gemm<double>(c.stream, side ? 'C' : 'N', 'N', p.n, m, p.n, cx(1.0, 0.0), A, p.A.ld, 0, X, m, 0,
                 czero<double>(), Out, m, 0, 1);
}

void apply_B(Ctx& c, Prob& p, int side, int m, const zd* X, zd* Out) {
    if (!p.hasB) {
        FH_HIP(hipMemcpyAsync(Out, X, sizeof(zd) * (size_t)p.n * m, hipMemcpyDeviceToDevice, c.stream));
        return;
    }
    const zd* B = (const zd*)p.B.val;
    gemm<double>(c.stream, side ? 'C' : 'N', 'N', p.n, m, p.n, cx(1.0, 0.0), B, p.B.ld, 0, X, m, 0,
                 czero<double>(), Out, m, 0, 1);
}

// ---------------------------------------------------------------------------
// dense contour filter (step 1): one LU per node, 'N' and 'C' solves
// ---------------------------------------------------------------------------
static void dense_factor(Ctx& c, Prob& p, int ne, const cplx* z, const fh_opts& o, fh_report* rep) {
    const int n = p.n;
    bool reuse = o.save_factors && (int)p.fact_z.size() == ne;
    if (reuse)
        for (int j = 0; j < ne; ++j) reuse = reuse && (p.fact_z[j] == z[j]);
    if (reuse) return;
    p.fact_z.clear();
    zd* M = (zd*)p.lu.ensure(sizeof(zd) * (size_t)ne * n * n);
    int* ipiv = (int*)p.ipiv.ensure(sizeof(int) * (size_t)ne * n);
    int* info = (int*)p.info.ensure(sizeof(int) * ne);
    zd* zd_ = (zd*)c.fb.zdev.ensure(sizeof(zd) * ne);
    to_dev(c, zd_, reinterpret_cast<const zd*>(z), ne);
    form_shift(c.stream, n, (const zd*)p.A.val, p.A.ld, p.hasB ? (const zd*)p.B.val : nullptr, p.B.ld, ne, zd_, M);
    lu_factor(c.stream, n, M, ne, ipiv, info, c.partial);
    std::vector<int> hinfo(ne);
    to_host(c, hinfo.data(), info, ne);
    if (rep) rep->n_factor += ne;
    for (int j = 0; j < ne; ++j)
        if (hinfo[j] != 0) {
            if (rep) rep->bad_node = j;
            throw Error(FH_SINGULAR_SHIFT, "zero pivot in the LU of (z_j B - A) at node " + std::to_string(j));
        }
    p.fact_z.assign(z, z + ne);
}


void filter(Ctx& c, Prob& p, int ne, const cplx* z, const cplx* w, int m0, const zd* Y, const zd* Yh, zd* Q,
            zd* Qh, const fh_opts& o, fh_report* rep, const cplx* lam, const int* cpart) {
    auto t0 = std::chrono::steady_clock::now();
    if (!p.dense) {
        sparse_filter(c, p, ne, z, w, m0, Y, Yh, Q, Qh, o, rep, lam, cpart);
    } else if (o.precision == FH_PREC_MIXED) {
        dense_filter_group(c, p, ne, z, w, m0, Y, Yh, Q, Qh, o, rep);
    } else {
        const int n = p.n;
        const size_t blk = (size_t)n * m0;
        dense_factor(c, p, ne, z, o, rep);
        FilterBufs& b = c.fb;
        zd* X = (zd*)b.X.ensure(sizeof(zd) * blk * ne);
        zd* Xh = (zd*)b.Xh.ensure(sizeof(zd) * blk * ne);
        zd* R = (zd*)b.R.ensure(sizeof(zd) * blk);
        zd* Rh = (zd*)b.Rh.ensure(sizeof(zd) * blk);
        zd* wd = (zd*)b.wdev.ensure(sizeof(zd) * ne);
        to_dev(c, wd, reinterpret_cast<const zd*>(w), ne);
        apply_B(c, p, 0, m0, Y, R);        // B Y
        apply_B(c, p, 1, m0, Yh, Rh);      // B^H Yh
        replicate<double>(c.stream, blk, R, X, ne);
        replicate<double>(c.stream, blk, Rh, Xh, ne);
        const zd* M = (const zd*)p.lu.p;
        const int* ipiv = (const int*)p.ipiv.p;
        lu_solve(c.stream, 'N', n, M, ipiv, m0, X, ne);     // (z_j B - A) Q_j = B Y
        lu_solve(c.stream, 'C', n, M, ipiv, m0, Xh, ne);    // (z_j B - A)^H Qh_j = B^H Yh
        accumulate(c.stream, ne, blk, X, blk, wd, false, Q);
        accumulate(c.stream, ne, blk, Xh, blk, wd, true, Qh);
        if (rep) rep->n_solve += 2 * ne;
        sync(c);
    }
    if (rep)
        rep->t_filter_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// dense shifted solves: one LU of (z_s B - A) per system, 'N' solves for the
// right systems (first nright), 'C' solves for the left ones
void dense_shifted_solve(Ctx& c, Prob& p, int nsys, int nright, const cplx* z, int m, const zd* B, zd* X,
                         const fh_opts& o, fh_report* rep) {
    const int n = p.n;
    const size_t blk = (size_t)n * m;
    dense_factor(c, p, nsys, z, o, rep);
    FH_HIP(hipMemcpyAsync(X, B, sizeof(zd) * blk * nsys, hipMemcpyDeviceToDevice, c.stream));
    const zd* M = (const zd*)p.lu.p;
    const int* ipiv = (const int*)p.ipiv.p;
    if (nright > 0) lu_solve(c.stream, 'N', n, M, ipiv, m, X, nright);
    if (nsys > nright)
        lu_solve(c.stream, 'C', n, M + (size_t)nright * n * n, ipiv + (size_t)nright * n, m, X + nright * blk,
                 nsys - nright);
    if (rep) rep->n_solve += nsys;
    sync(c);
}

// ---------------------------------------------------------------------------
// FEAST (complete algorithm figure)
// ---------------------------------------------------------------------------

// One FEAST run (complete algorithm figure) as a state machine: the caller
// fills Q and Qh by the contour filter (step 1) from Ycur / Yhcur, then
// step() performs steps 2-5; finish() writes the outputs (step 5.d).
struct FeastRun {
    Ctx& c;
    Prob& p;
    fh_contour ct;
    fh_opts o;
    fh_report* rep;
    FeastBufs& B;
    std::vector<cplx> z, w;
    int n, m0in, ne;
    double alpha;
    zd *Ycur, *Yhcur, *Q, *Qh, *U, *Uh, *T1, *T2, *T3, *T4, *BQ, *S, *Sh, *gam, *AUr, *BUr, *lam, *W, *Wh;
    double *num, *den, *num2, *den2;
    int *ints, *perm;
    int mcur = 0, it = 0, info = FH_NOT_CONVERGED, m_s = 0, prev_nconv = -1;
    bool converged = false, prev_pass = false, done = false;
    const bool force_bq_retry = [] {
        const char* e = std::getenv("FH_TEST_BQ_REVERSED");
        return e && e[0] == '1';
    }();
    std::vector<cplx> rho_prev, hlam, hbq, rho;
    std::vector<char> inside_prev, inside;
    std::vector<double> res, hn, hd, hn2, hd2;
    std::vector<int> sel;
    std::chrono::steady_clock::time_point t0;

    FeastRun(Ctx& c_, Prob& p_, FeastBufs& bufs, const fh_contour& ct_, const cplx* zin, const cplx* win,
             const fh_opts& o_, const zd* Yio, const zd* Yhio, const zd* lambda, fh_report* rep_)
        : c(c_), p(p_), ct(ct_), o(o_), rep(rep_), B(bufs) {
        n = p.n;
        m0in = o.m0;
        ne = ct.ne;
        if (zin) { z.assign(zin, zin + ne); w.assign(win, win + ne); }
        else contour_nodes(ct, z, w);
        alpha = contour_alpha(ct);
        const size_t big = (size_t)n * m0in, sm = (size_t)m0in * m0in;
        Ycur = (zd*)B.Ycur.ensure(sizeof(zd) * big);
        Yhcur = (zd*)B.Yhcur.ensure(sizeof(zd) * big);
        Q = (zd*)B.Q.ensure(sizeof(zd) * big);
        Qh = (zd*)B.Qh.ensure(sizeof(zd) * big);
        U = (zd*)B.U.ensure(sizeof(zd) * big);
        Uh = (zd*)B.Uh.ensure(sizeof(zd) * big);
        T1 = (zd*)B.T1.ensure(sizeof(zd) * big);
        T2 = (zd*)B.T2.ensure(sizeof(zd) * big);
        T3 = (zd*)B.T3.ensure(sizeof(zd) * big);
        T4 = (zd*)B.T4.ensure(sizeof(zd) * big);
        BQ = (zd*)B.BQ.ensure(sizeof(zd) * sm);
        S = (zd*)B.S.ensure(sizeof(zd) * sm);
        Sh = (zd*)B.Sh.ensure(sizeof(zd) * sm);
        gam = (zd*)B.gam.ensure(sizeof(zd) * m0in);
        AUr = (zd*)B.AUr.ensure(sizeof(zd) * sm);
        BUr = (zd*)B.BUr.ensure(sizeof(zd) * sm);
        lam = (zd*)B.lam.ensure(sizeof(zd) * m0in);
        W = (zd*)B.W.ensure(sizeof(zd) * sm);
        Wh = (zd*)B.Wh.ensure(sizeof(zd) * sm);
        num = (double*)B.num.ensure(sizeof(double) * m0in);
        den = (double*)B.den.ensure(sizeof(double) * m0in);
        num2 = (double*)B.num2.ensure(sizeof(double) * m0in);
        den2 = (double*)B.den2.ensure(sizeof(double) * m0in);
        ints = (int*)B.ints.ensure(sizeof(int) * 4);
        perm = (int*)B.perm.ensure(sizeof(int) * m0in);
        // step 0: start subspaces
        FH_HIP(hipMemcpyAsync(Ycur, Yio, sizeof(zd) * big, hipMemcpyDeviceToDevice, c.stream));
        FH_HIP(hipMemcpyAsync(Yhcur, Yhio, sizeof(zd) * big, hipMemcpyDeviceToDevice, c.stream));
        mcur = m0in;
        hlam.assign(m0in, 0.0);
        hbq.assign(sm, 0.0);
        rho.assign(m0in, 0.0);
        inside.assign(m0in, 0);
        res.assign(m0in, 0.0);
        hn.assign(m0in, 0.0);
        hd.assign(m0in, 0.0);
        hn2.assign(m0in, 0.0);
        hd2.assign(m0in, 0.0);
        // resume: the start columns are Ritz vectors whose values are passed in lambda
        if (o.resume) to_host(c, reinterpret_cast<zd*>(hlam.data()), lambda, m0in);
        // conj_pairs = 2: a real start block (its imaginary part dropped) makes
        // every later subspace closed under conjugation
        half = sparse_conj_closed(p, ne, z.data(), w.data(), o);
        if (half && !o.resume) {
            real_part(c.stream, (long)big, Ycur);
            real_part(c.stream, (long)big, Yhcur);
        }
    }

    // Ritz values of the current columns (residual form of the iterative
    // filter from the second iteration on), or nullptr
    const cplx* filter_lambda() const {
        if (!((it >= 1 || o.resume) && !p.dense)) return nullptr;
        return half ? flam.data() : hlam.data();
    }

    // conj_pairs = 2 (real CSR matrix, nodes in conjugate pairs): before each
    // filter, pair the Ritz values as conjugates and make the pairs exact,
    // x_k = conj(x_i), xh_k = conj(xh_i), lambda_k = conj(lambda_i), and the
    // vectors of real Ritz values real.  In exact arithmetic the subspace of a
    // real start block stays closed under conjugation, so this changes the
    // columns by rounding only; the filter then solves n_e/2 nodes per side.
    // Returns the column partners, or nullptr when the mode is off.
    bool half = false;
    std::vector<int> cpart;
    std::vector<cplx> flam;
    DBuf cpdev;
    const int* prepare_filter() {
        if (!half) return nullptr;
        const int m = mcur;
        if (!filter_lambda_needed()) {
            cpart.resize(m);
            std::iota(cpart.begin(), cpart.end(), 0);   // real start block
            return cpart.data();
        }
        cpart = conj_partners(hlam.data(), m);
        flam.assign(hlam.begin(), hlam.begin() + m);
        for (int i = 0; i < m; ++i) {
            const int k = cpart[i];
            if (k == i && std::isfinite(flam[i].real())) flam[i] = cplx(flam[i].real(), 0.0);
            else if (k > i) flam[k] = std::conj(flam[i]);
        }
        int* d = (int*)cpdev.ensure(sizeof(int) * m);
        to_dev(c, d, cpart.data(), m);
        conj_close_cols(c.stream, n, m, Ycur, Yhcur, d, c.partial);
        return cpart.data();
    }
    bool filter_lambda_needed() const { return it >= 1 || o.resume; }

    // Steps 2-5 of iteration it+1 (Q, Qh filled), in phases so that many runs
    // can share one launch of each small eigensolver: GPU work is enqueued by
    // the launch_* / phase_bq calls, host decisions read results in read_* /
    // decide.  step() runs them for this run alone.
    DBuf eigw;
    int mt = 0;

    EigJob job_biortho() {
        return EigJob{mcur, 1e-16, BQ, nullptr, gam, S, Sh, ints, ints + 1,
                      (zd*)eigw.ensure(eig_work_size(m0in))};
    }
    EigJob job_reduced() {
        return EigJob{mt, 0.0, AUr, BUr, lam, W, Wh, ints + 2, nullptr, (zd*)eigw.ensure(eig_work_size(m0in))};
    }

    // step 2.a: B_Q = Qh^H B Q
    // Products of steps 2-5.  The batched driver sets gN / gC: dense products
    // are then appended to these lists (op(A) = A, resp. A^H) and launched by
    // it as one grouped GEMM over all runs; otherwise they launch here.
    std::vector<GItem<double>>* gN = nullptr;
    std::vector<GItem<double>>* gC = nullptr;
    // C (M x N, ld ldc) = op(A) B, op 'N' or 'C', row-major
    void prod(char op, int M, int N, int K, const zd* A, long lda, const zd* B, long ldb, zd* C, long ldc) {
        std::vector<GItem<double>>* sink = op == 'C' ? gC : gN;
        if (sink) {
            sink->push_back(GItem<double>{A, B, C, M, N, K, (int)lda, (int)ldb, (int)ldc, 0, 0, cx(1.0, 0.0), 0});
            return;
        }
        gemm<double>(c.stream, op, 'N', M, N, K, cx(1.0, 0.0), A, lda, 0, B, ldb, 0, czero<double>(), C, ldc, 0, 1);
    }
    // op(A) X or op(B) X of this run's problem (side 1: conjugate transpose)
    void prod_A(int side, int m, const zd* X, zd* Out) {
        if (!p.dense) { apply_A(c, p, side, m, X, Out); return; }
        prod(side ? 'C' : 'N', n, m, n, (const zd*)p.A.val, p.A.ld, X, m, Out, m);
    }
    // returns the operand that holds op(B) X (X itself when B = I)
    const zd* prod_B(int side, int m, const zd* X, zd* Out) {
        if (!p.hasB) return X;
        if (!p.dense) { apply_B(c, p, side, m, X, Out); return Out; }
        prod(side ? 'C' : 'N', n, m, n, (const zd*)p.B.val, p.B.ld, X, m, Out, m);
        return Out;
    }

    const zd* BQin = nullptr;
    void phase_bq_a() {   // B Q
        ++it;
        BQin = prod_B(0, mcur, Q, T1);
    }
    void phase_bq_b() { gemm_hn_tall(c.stream, n, mcur, mcur, Qh, mcur, BQin, mcur, BQ, mcur, c.partial); }
    void phase_bq() {
        phase_bq_a();
        phase_bq_b();
    }

    // The shifted QR iteration on B_Q ran out of its iteration budget (code 1).
    // Its convergence depends on the order of the basis vectors, not only on
    // the spectrum: run it once more on the reversed order J B_Q J (J the
    // exchange matrix; same eigenvalues, eigenvectors J v), then reverse the
    // rows of S and Sh so that they refer to the columns of Q and Qh again.
    // AUr is free at this point of the iteration (steps 3.e-3.f fill it).
    void retry_bq_reversed(int* hi) {
        const int m = mcur;
        if (rep) ++rep->n_bq_retry;
        std::vector<cplx> rb((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) rb[(size_t)i * m + j] = hbq[(size_t)(m - 1 - i) * m + (m - 1 - j)];
        to_dev(c, AUr, reinterpret_cast<const zd*>(rb.data()), rb.size());
        eig_biortho(c.stream, m, AUr, 1e-16, gam, S, Sh, ints, ints + 1, eigw);
        to_host(c, hi, ints, 2);
        if (hi[1] != 0) return;
        for (zd* M : {S, Sh}) {
            to_host(c, rb.data(), M, rb.size());
            for (int i = 0; i < m / 2; ++i)
                std::swap_ranges(rb.begin() + (size_t)i * m, rb.begin() + (size_t)(i + 1) * m,
                                 rb.begin() + (size_t)(m - 1 - i) * m);
            to_dev(c, M, reinterpret_cast<const zd*>(rb.data()), rb.size());
        }
    }

    // after steps 3.a-3.c (eig_biortho): spurious test (2.b), resize count
    void read_bq() {
        to_host(c, hbq.data(), BQ, (size_t)mcur * mcur);
        m_s = 0;
        if (it >= 2) {
            for (int i = 0; i < mcur; ++i) {
                const cplx r2 = rho_prev[i] * rho_prev[i];
                const double rel = std::abs(r2 - hbq[(size_t)i * mcur + i]) / std::abs(r2);
                const bool flag = !(rel < 0.1);
                if (flag && inside_prev[i]) ++m_s;
            }
        }
        int hi[2];
        to_host(c, hi, ints, 2);
        // FH_TEST_BQ_REVERSED=1 (test switch) takes the retry at every
        // iteration, so that its row reversal of S and Sh is exercised
        if (hi[1] == 1 || (hi[1] == 0 && force_bq_retry)) retry_bq_reversed(hi);
        if (hi[1] != 0) {
            // diagnostics: FH_DUMP_BQ=<path> writes the matrix whose
            // eigendecomposition failed (m, then m x m complex row-major)
            if (const char* path = std::getenv("FH_DUMP_BQ")) {
                if (FILE* f = std::fopen(path, "wb")) {
                    const int mm = mcur;
                    std::fwrite(&mm, sizeof(int), 1, f);
                    std::fwrite(hbq.data(), sizeof(cplx), (size_t)mcur * mcur, f);
                    std::fclose(f);
                }
            }
            throw Error(FH_EIG_FAILED, "eigendecomposition of B_Q failed (code " + std::to_string(hi[1]) + ")");
        }
        mt = hi[0];
        FH_REQUIRE(mt >= 1 && mt <= mcur, FH_EIG_FAILED, "resize produced an empty subspace");
    }

    // step 3.d: U = Q S, Uh = Qh Sh
    void launch_rr_a() {
        prod('N', n, mt, mcur, Q, mcur, S, mcur, U, mt);        // S, Sh: mcur x mcur (first mt columns used)
        prod('N', n, mt, mcur, Qh, mcur, Sh, mcur, Uh, mt);
    }
    // step 4.a, products with the operators
    const zd* BUin = nullptr;
    void launch_rr_b() {
        prod_A(0, mt, U, T1);
        BUin = prod_B(0, mt, U, T2);
    }
    // step 4.a: A_U = Uh^H A U, B_U = Uh^H B U
    void launch_rr_c() {
        gemm_hn_tall(c.stream, n, mt, mt, Uh, mt, T1, mt, AUr, mt, c.partial);
        gemm_hn_tall(c.stream, n, mt, mt, Uh, mt, BUin, mt, BUr, mt, c.partial);
    }
    void launch_rr() {
        launch_rr_a();
        launch_rr_b();
        launch_rr_c();
    }

    // after step 4.b (eig_reduced): Ritz values, step 4.c
    void read_lam() {
        int e4 = 0;
        to_host(c, &e4, ints + 2, 1);
        if (e4 != 0) throw Error(FH_EIG_FAILED, "reduced eigenproblem failed (code " + std::to_string(e4) + ")");
        to_host(c, reinterpret_cast<zd*>(hlam.data()), lam, mt);
        for (int i = 0; i < mt; ++i) rho[i] = rational(ne, z.data(), w.data(), hlam[i]);
    }

    // step 4.d: Y = U W, Yh = Uh Wh
    void launch_ritz_a() {
        prod('N', n, mt, mt, U, mt, W, mt, Ycur, mt);
        prod('N', n, mt, mt, Uh, mt, Wh, mt, Yhcur, mt);
    }
    // products of step 5.b: A Y, B Y, A^H Yh, B^H Yh
    const zd *BY = nullptr, *BhYh = nullptr;
    void launch_ritz_b() {
        prod_A(0, mt, Ycur, T1);
        BY = prod_B(0, mt, Ycur, T2);
        prod_A(1, mt, Yhcur, T3);
        BhYh = prod_B(1, mt, Yhcur, T4);
    }
    // step 5.b: residual norms of the right and left pairs
    void launch_ritz_c() {
        res_colnorms(c.stream, n, mt, T1, BY, mt, lam, false, num, den, c.partial);
        res_colnorms(c.stream, n, mt, T3, BhYh, mt, lam, true, num2, den2, c.partial2);
    }
    void launch_ritz() {
        launch_ritz_a();
        launch_ritz_b();
        launch_ritz_c();
    }

    // steps 5.a-5.c; true when the run is over
    bool decide() {
        to_host(c, hn.data(), num, mt);
        to_host(c, hd.data(), den, mt);
        to_host(c, hn2.data(), num2, mt);
        to_host(c, hd2.data(), den2, mt);
        int m_r = 0;
        for (int i = 0; i < mt; ++i) {
            double r1 = hn[i] / (alpha * hd[i]), r2 = hn2[i] / (alpha * hd2[i]);
            double r = std::max(r1, r2);
            if (!std::isfinite(r)) r = INFINITY;
            res[i] = r;
            inside[i] = inside_contour(ct, hlam[i]);   // step 5.a
            m_r += inside[i];
        }
        // step 5.c: the m = m_r - m_s smallest inside residuals below eps
        const int m = m_r - m_s;
        sel.clear();
        for (int i = 0; i < mt; ++i)
            if (inside[i]) sel.push_back(i);
        std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) { return res[a] < res[b]; });
        if (m > 0) sel.resize(m);
        else sel.clear();
        converged = m > 0;
        for (int i : sel) converged = converged && (res[i] < o.eps);
        if (o.confirm == 1) {
            // optional stricter exit (not the paper's rule): an exit that relies
            // on spurious flags (some inside pair above eps, passed over as
            // flagged) must be confirmed by the next iteration with the same
            // number of converged inside pairs; when every inside pair meets
            // eps the flags exclude nothing and the exit is immediate
            int nconv = 0;
            for (int i = 0; i < mt; ++i) nconv += (inside[i] && res[i] < o.eps) ? 1 : 0;
            const bool all_in = m_r > 0 && nconv == m_r;
            const bool passed = converged;
            if (converged && m_s > 0 && !all_in && !(prev_pass && prev_nconv == nconv)) converged = false;
            prev_pass = passed;
            prev_nconv = nconv;
        }
        mcur = mt;
        if (verbose()) {
            double worst = 0.0;
            for (int i : sel) worst = std::max(worst, res[i]);
            std::fprintf(stderr,
                         "[feasthip] it %d m0 %d m_r %d m_s %d worst-res %.3e filter %.1f ms iter %.1f ms inner-steps %lld "
                         "inner-relres %.2e\n",
                         it, mt, m_r, m_s, worst, rep ? rep->t_filter_ms : 0.0,
                         std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count(),
                         rep ? rep->inner_steps : 0LL, rep ? rep->inner_relres : 0.0);
            std::fflush(stderr);
        }
        if (rep) {
            rep->iters = it;
            rep->m0_final = mt;
            rep->m_s = m_s;
            rep->m = (int)sel.size();
            rep->t_iter_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        if (converged) {
            info = FH_OK;
            done = true;
            return true;
        }
        rho_prev.assign(rho.begin(), rho.begin() + mt);
        inside_prev.assign(inside.begin(), inside.begin() + mt);
        if (it == o.max_iter) {
            // every one of the m0 Ritz values inside: m0 is probably not above
            // the number of eigenvalues inside (the method needs m0 >= m)
            info = (m_r == 0) ? FH_NO_EIG_INSIDE : (m_r >= m0in ? FH_M0_TOO_SMALL : FH_NOT_CONVERGED);
            done = true;
            return true;
        }
        return false;
    }

    bool step() {
        phase_bq();
        const EigJob jb = job_biortho();
        eig_biortho(c.stream, jb.m, jb.in1, jb.eta, jb.out0, jb.out1, jb.out2, jb.i0, jb.i1, eigw);
        read_bq();
        launch_rr();
        const EigJob jr = job_reduced();
        eig_reduced(c.stream, jr.m, jr.in1, jr.in2, jr.out0, jr.out1, jr.out2, jr.i0, eigw);
        read_lam();
        launch_ritz();
        return decide();
    }

    // step 5.d: the m = m_r - m_s converged pairs of step 5.c (the m smallest
    // inside residuals) in the first m columns, sorted by (Re, Im).  With
    // opts.confirm (1 or 2) every inside pair whose residual meets eps is
    // returned.
    // The remaining Ritz vectors follow in columns m..m0_final-1 so that the
    // whole search subspace can be reused as a start (resume).
    int finish(zd* Yio, zd* Yhio, zd* lambda, double* res_out) {
        if (converged && o.confirm) {
            for (int i = 0; i < mcur; ++i)
                if (inside[i] && res[i] < o.eps && std::find(sel.begin(), sel.end(), i) == sel.end()) sel.push_back(i);
        }
        std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) {
            if (hlam[a].real() != hlam[b].real()) return hlam[a].real() < hlam[b].real();
            return hlam[a].imag() < hlam[b].imag();
        });
        const int m_out = converged ? (int)sel.size() : 0;
        std::vector<int> order(sel.begin(), sel.end());
        for (int i = 0; i < mcur; ++i)
            if (std::find(order.begin(), order.end(), i) == order.end()) order.push_back(i);
        to_dev(c, perm, order.data(), mcur);
        gather_cols(c.stream, n, mcur, Ycur, mcur, perm, Yio, m0in);
        gather_cols(c.stream, n, mcur, Yhcur, mcur, perm, Yhio, m0in);
        std::vector<cplx> lo(mcur);
        for (int k = 0; k < mcur; ++k) lo[k] = hlam[order[k]];
        to_dev(c, lambda, reinterpret_cast<const zd*>(lo.data()), mcur);
        if (res_out)
            for (int k = 0; k < mcur; ++k) res_out[k] = res[order[k]];
        sync(c);
        if (rep) {
            rep->m = m_out;
            rep->info = info;
        }
        return info;
    }
};

int feast(Ctx& c, Prob& p, const fh_contour& ct, const cplx* zin, const cplx* win, const fh_opts& o, zd* Yio,
          zd* Yhio, zd* lambda, double* res_out, fh_report* rep) {
    FeastRun r(c, p, c.sb, ct, zin, win, o, Yio, Yhio, lambda, rep);
    for (;;) {
        r.t0 = std::chrono::steady_clock::now();
        // step 1: contour integration
        const int* cp = r.prepare_filter();
        filter(c, p, r.ne, r.z.data(), r.w.data(), r.mcur, r.Ycur, r.Yhcur, r.Q, r.Qh, o, rep, r.filter_lambda(), cp);
        if (r.step()) break;
    }
    return r.finish(Yio, Yhio, lambda, res_out);
}

// Many dense instances at once: the contour filters of all instances (every
// node, both sides) run through one grouped engine per iteration, factors
// computed once for all instances; steps 2-5 run per instance.
int feast_batched(Ctx& c, int count, Prob* const* probs, const fh_contour* cts, const fh_opts& o, zd* const* Y,
                  zd* const* Yh, zd* const* lambda, double* const* res, fh_report* reps) {
    hipStream_t st = c.stream;
    std::vector<std::unique_ptr<FeastBufs>> bufs;
    std::vector<std::unique_ptr<FeastRun>> runs;
    std::vector<Prob*> plist(probs, probs + count);
    std::vector<std::vector<cplx>> zs;
    for (int i = 0; i < count; ++i) {
        bufs.emplace_back(new FeastBufs());
        if (reps) std::memset(&reps[i], 0, sizeof(fh_report));
        runs.emplace_back(new FeastRun(c, *probs[i], *bufs[i], cts[i], nullptr, nullptr, o, Y[i], Yh[i], lambda[i],
                                       reps ? &reps[i] : nullptr));
        zs.push_back(runs[i]->z);
    }
    DenseGroup G;
    DBuf jobbuf;
    // the dense products of steps 1-5 of all runs as grouped GEMMs, one launch
    // per dependent stage (each plan's work list is used once per iteration)
    std::vector<GItem<double>> gn, gc;
    GroupPlan<double> gp[12];
    auto grouped = [&](GroupPlan<double>& pn, GroupPlan<double>& pc) {
        if (!gn.empty()) { group_gemm_plan(pn, false, gn, GTILE_64); pn.run(st); gn.clear(); }
        if (!gc.empty()) { group_gemm_plan(pc, true, gc, GTILE_64); pc.run(st); gc.clear(); }
    };
    std::vector<const zd*> bys(count), bhys(count);
    fh_report frep{};
    dg_build(c, G, plist, zs, o.precision == FH_PREC_MIXED, &frep);
    std::vector<int> first(count);   // first system of each instance
    for (int i = 0, s = 0; i < count; ++i) {
        first[i] = s;
        s += cts[i].ne;
    }
    std::vector<DBuf> wdev(count);
    for (int i = 0; i < count; ++i) {
        zd* wd = (zd*)wdev[i].ensure(sizeof(zd) * cts[i].ne);
        to_dev(c, wd, reinterpret_cast<const zd*>(runs[i]->w.data()), cts[i].ne);
        if (reps) reps[i].n_factor = cts[i].ne;
    }
    for (;;) {
        std::vector<int> m(G.count, 0);
        int active = 0;
        for (int i = 0; i < count; ++i) {
            if (runs[i]->done) continue;
            ++active;
            for (int j = 0; j < cts[i].ne; ++j) m[first[i] + j] = runs[i]->mcur;
        }
        if (!active) break;
        auto t0 = std::chrono::steady_clock::now();
        dg_layout(c, G, m);
        // right-hand sides B Y_i and B^H Yh_i, replicated over the nodes of instance i
        for (int i = 0; i < count; ++i) {
            FeastRun& r = *runs[i];
            if (r.done) continue;
            r.t0 = t0;
            r.gN = &gn;
            r.gC = &gc;
            bys[i] = r.prod_B(0, r.mcur, r.Ycur, r.T1);
            bhys[i] = r.prod_B(1, r.mcur, r.Yhcur, r.T2);
            r.gN = r.gC = nullptr;
        }
        grouped(gp[8], gp[9]);
        for (int i = 0; i < count; ++i) {
            FeastRun& r = *runs[i];
            if (r.done) continue;
            const long blk = (long)r.n * r.mcur;
            const long off = G.voff[first[i]];
            replicate<double>(st, blk, bys[i], (zd*)G.Bv.p + off, r.ne);
            replicate<double>(st, blk, bhys[i], (zd*)G.Bhv.p + off, r.ne);
        }
        fh_report srep{};
        dg_solve(c, G, o, &srep);
        // systems solved again with FP64 factors, attributed to their problems
        if (reps && srep.n_fallback > 0)
            for (int s : G.fb_sys)
                for (int i = 0; i < count; ++i)
                    if (s >= first[i] && s < first[i] + cts[i].ne) reps[i].n_fallback += 1;
        for (int i = 0; i < count; ++i) {
            FeastRun& r = *runs[i];
            if (r.done) continue;
            const long blk = (long)r.n * r.mcur;
            const long off = G.voff[first[i]];
            accumulate(st, r.ne, blk, (const zd*)G.Xv.p + off, blk, (const zd*)wdev[i].p, false, r.Q);
            accumulate(st, r.ne, blk, (const zd*)G.Xhv.p + off, blk, (const zd*)wdev[i].p, true, r.Qh);
        }
        sync(c);
        const double tf = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::vector<FeastRun*> act;
        for (int i = 0; i < count; ++i) {
            FeastRun& r = *runs[i];
            if (r.done) continue;
            if (reps) {
                reps[i].n_solve += 2 * r.ne;
                reps[i].t_filter_ms = tf;
                reps[i].inner_steps = srep.inner_steps;
                reps[i].inner_relres = srep.inner_relres;
            }
            act.push_back(&r);
        }
        // steps 2-5 of all active runs in lockstep: one launch of each small
        // eigensolver for all of them, host decisions between
        std::vector<EigJob> jobs(act.size());
        EigJob* dj = (EigJob*)jobbuf.ensure(sizeof(EigJob) * std::max<size_t>(1, act.size()));
        for (FeastRun* r : act) { r->gN = &gn; r->gC = &gc; }
        for (FeastRun* r : act) r->phase_bq_a();
        grouped(gp[10], gp[11]);
        for (FeastRun* r : act) r->phase_bq_b();
        for (size_t k = 0; k < act.size(); ++k) jobs[k] = act[k]->job_biortho();
        to_dev(c, dj, jobs.data(), jobs.size());
        int mmax = 1;
        for (const EigJob& jj : jobs) mmax = std::max(mmax, jj.m);
        eig_biortho_batched(st, (int)act.size(), dj, mmax);
        for (FeastRun* r : act) r->read_bq();
        for (FeastRun* r : act) r->launch_rr_a();
        grouped(gp[0], gp[1]);
        for (FeastRun* r : act) r->launch_rr_b();
        grouped(gp[2], gp[3]);
        for (FeastRun* r : act) r->launch_rr_c();
        for (size_t k = 0; k < act.size(); ++k) jobs[k] = act[k]->job_reduced();
        to_dev(c, dj, jobs.data(), jobs.size());
        mmax = 1;
        for (const EigJob& jj : jobs) mmax = std::max(mmax, jj.m);
        eig_reduced_batched(st, (int)act.size(), dj, mmax);
        for (FeastRun* r : act) r->read_lam();
        for (FeastRun* r : act) r->launch_ritz_a();
        grouped(gp[4], gp[5]);
        for (FeastRun* r : act) r->launch_ritz_b();
        grouped(gp[6], gp[7]);
        for (FeastRun* r : act) r->launch_ritz_c();
        for (FeastRun* r : act) { r->gN = nullptr; r->gC = nullptr; }
        for (FeastRun* r : act) r->decide();
    }
    int worst = FH_OK;
    for (int i = 0; i < count; ++i) {
        const int inf = runs[i]->finish(Y[i], Yh[i], lambda[i], res ? res[i] : nullptr);
        if (inf != FH_OK && worst == FH_OK) worst = inf;
    }
    return worst;
}

}  // namespace fh
