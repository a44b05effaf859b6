// Small dense non-Hermitian eigenproblems of the Rayleigh-Ritz steps, in
// FP64 on the GPU, one workgroup per problem:
//   * step 3.a: B_Q = V Gamma Vh^H (Vh = V^{-H}), then 3.b-3.c: stable sort by
//     decreasing |gamma|, resize count, and the bi-orthonormalizing factors of
//     eq:uu;
//   * step 4.b: A_U W = B_U W Lambda with Wh^H B_U W = I, solved as the
//     standard problem C = B_U^{-1} A_U (B_U is close to I after the
//     B-bi-orthonormalization); the left vectors follow from Wh^H = W^{-1} B_U^{-1}.
// Algorithms (textbook): Householder reduction to Hessenberg form, complex
// single-shift QR with Wilkinson shifts and deflation to the Schur form,
// eigenvectors by back substitution on the triangular factor, inverses by
// Gauss-Jordan elimination with partial pivoting.  All matrices row-major,
// held in a global scratch buffer that stays resident in L1/L2.
#include <cfloat>

#include "fh_kernels.h"

namespace fh {

constexpr int ENT = 256;

__device__ double block_sum(double v, double* red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = ENT / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// Householder reduction H <- Q^H H Q, Z <- Z Q (Z must hold I or a prior basis)
__device__ void hessenberg(int m, zd* H, zd* Z, zd* v, double* red) {
    const int tid = threadIdx.x;
    for (int k = 0; k < m - 2; ++k) {
        double part = 0.0;
        for (int i = k + 2 + tid; i < m; i += ENT) part += abs2(H[(long)i * m + k]);
        const double sigma2 = block_sum(part, red);
        if (sigma2 == 0.0) continue;
        const zd alpha = H[(long)(k + 1) * m + k];
        const double aa = cabs(alpha);
        const double xnorm = sqrt(aa * aa + sigma2);
        const zd ph = aa > 0.0 ? cx(alpha.re / aa, alpha.im / aa) : cx(1.0, 0.0);
        const zd beta = cx(-xnorm * ph.re, -xnorm * ph.im);
        const zd v0 = (aa + xnorm) * ph;
        const double tau = 2.0 / (abs2(v0) + sigma2);
        const int len = m - k - 1;
        for (int i = tid; i < len; i += ENT) v[i] = (i == 0) ? v0 : H[(long)(k + 1 + i) * m + k];
        __syncthreads();
        for (int j = k + tid; j < m; j += ENT) {           // left: H <- (I - tau v v^H) H
            zd s = czero<double>();
            for (int i = 0; i < len; ++i) cfma_conj(s, v[i], H[(long)(k + 1 + i) * m + j]);
            s = tau * s;
            for (int i = 0; i < len; ++i) cfms(H[(long)(k + 1 + i) * m + j], v[i], s);
        }
        __syncthreads();
        for (int i = tid; i < 2 * m; i += ENT) {             // right: X <- X (I - tau v v^H)
            zd* R = (i < m) ? (H + (long)i * m) : (Z + (long)(i - m) * m);
            zd t = czero<double>();
            for (int l = 0; l < len; ++l) cfma(t, R[k + 1 + l], v[l]);
            t = tau * t;
            for (int l = 0; l < len; ++l) cfms(R[k + 1 + l], t, conj(v[l]));
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < m; i += ENT) H[(long)i * m + k] = (i == k + 1) ? beta : czero<double>();
        __syncthreads();
    }
}

// complex Givens: [c s; -conj(s) c] [x; y] = [r; 0], c real
__device__ __forceinline__ void givens(zd x, zd y, double& c, zd& s, zd& r) {
    const double ax = cabs(x), ay = cabs(y);
    if (ay == 0.0) { c = 1.0; s = czero<double>(); r = x; }
    else if (ax == 0.0) { c = 0.0; s = cx(y.re / ay, -y.im / ay); r = cx(ay, 0.0); }
    else {
        const double nrm = hypot(ax, ay);
        c = ax / nrm;
        const zd ph = cx(x.re / ax, x.im / ax);
        s = (1.0 / nrm) * (ph * conj(y));
        r = nrm * ph;
    }
}

// Shifted QR on an upper Hessenberg H to the Schur form T (in H), Z <- Z G^H.
// Returns 0 on success, 1 if the iteration budget is exhausted.  loose: the
// stagnation fallback below deflates at sqrt(ulp) ||H|| after 5 max(10, m)
// sweeps (B_Q), else at ulp ||H|| after 10 max(10, m) (reduced eigenproblem).
__device__ int schur_qr(int m, zd* H, zd* Z, bool loose) {
    const int tid = threadIdx.x;
    const double ulp = DBL_EPSILON, smlnum = DBL_MIN * (double(m) / DBL_EPSILON);
    int ihi = m - 1, its = 0;
    __shared__ int lsh, lst;
    // Frobenius norm of H (kept by every unitary similarity of the iteration):
    // after a number of sweeps without a deflation a subdiagonal entry below
    // tol ||H|| counts as negligible too.  The local test stalls for good on
    // a tight cluster: B_Q near convergence holds dozens of eigenvalues
    // rho_a^2 = 1 to within 1e-8 (the converged pairs), where the Wilkinson
    // shift cannot separate the trailing entry from its neighbours (seen
    // stuck at |h| = 1e-11 for 2,880 sweeps on the 64^3 workload).  B_Q's
    // decomposition only resizes and bi-orthonormalizes the subspace, and
    // the reduced eigenproblem restores Wh^H B_U W = I exactly, so deflating
    // at sqrt(ulp) ||H|| there costs no accuracy in the result; the reduced
    // eigenproblem itself keeps ulp ||H||.
    __shared__ double hred[ENT];
    {
        double a = 0.0;
        for (int e = tid; e < m * m; e += ENT) a += abs2(H[e]);
        hred[tid] = a;
        __syncthreads();
        for (int s2 = ENT / 2; s2 > 0; s2 >>= 1) {
            if (tid < s2) hred[tid] += hred[tid + s2];
            __syncthreads();
        }
    }
    const double hnorm = sqrt(hred[0]);
    const int stall = (loose ? 5 : 10) * max(10, m);
    const double stol = (loose ? sqrt(ulp) : ulp) * hnorm;
    __syncthreads();
    while (ihi >= 1) {
        // largest kk <= ihi with a negligible subdiagonal entry (0 if none):
        // every thread tests its own entries and one LDS maximum combines them
        // (a serial scan down from ihi costs one memory latency per entry)
        if (tid == 0) lsh = 0;
        __syncthreads();
        for (int kk = 1 + tid; kk <= ihi; kk += ENT) {
            const double sub = cabs1(H[(long)kk * m + kk - 1]);
            double tst = cabs1(H[(long)(kk - 1) * m + kk - 1]) + cabs1(H[(long)kk * m + kk]);
            if (tst == 0.0) {
                if (kk - 2 >= 0) tst += fabs(H[(long)(kk - 1) * m + kk - 2].re);
                if (kk + 1 <= ihi) tst += fabs(H[(long)(kk + 1) * m + kk].re);
            }
            if (sub <= fmax(ulp * tst, smlnum) || (its > stall && sub <= stol))
                atomicMax(&lsh, kk);
        }
        __syncthreads();
        const int l = lsh;
        if (l > 0 && tid == 0) H[(long)l * m + l - 1] = czero<double>();
        __syncthreads();
        if (l == ihi) { --ihi; its = 0; continue; }
        // shift: Wilkinson's, or every 10 iterations without a deflation an
        // exceptional one, alternating between the top and the bottom of the
        // active block (the schedule of LAPACK's complex QR iteration)
        zd mu;
        if (its > 0 && its % 20 == 10) {
            mu = H[(long)l * m + l] + cx(0.75 * fabs(H[(long)(l + 1) * m + l].re), 0.0);
        } else if (its > 0 && its % 20 == 0) {
            mu = H[(long)ihi * m + ihi] + cx(0.75 * fabs(H[(long)ihi * m + ihi - 1].re), 0.0);
        } else {
            const zd a = H[(long)(ihi - 1) * m + ihi - 1], b = H[(long)(ihi - 1) * m + ihi];
            const zd c = H[(long)ihi * m + ihi - 1], d = H[(long)ihi * m + ihi];
            const zd t2 = 0.5 * (a + d);
            const zd disc = csqrt(t2 * t2 - (a * d - b * c));
            const zd mu1 = t2 + disc, mu2 = t2 - disc;
            mu = (cabs(mu1 - d) <= cabs(mu2 - d)) ? mu1 : mu2;
        }
        // start row, as in LAPACK's complex QR: the lowest ks in (l, ihi) where
        // a sweep begun with the shift at row ks leaves H[ks][ks-1] negligible
        // (its fill-in is dropped).  On a graded H — B_Q once the filter has
        // suppressed part of the subspace — the sweep then stays in the small
        // trailing block instead of mixing rounding errors of the large block
        // into it, which would keep it from ever deflating.
        if (tid == 0) lst = l;
        __syncthreads();
        for (int M = l + 1 + tid; M < ihi; M += ENT) {
            const zd h11 = H[(long)M * m + M], h22 = H[(long)(M + 1) * m + M + 1];
            const double a11 = cabs1(h11 - mu), a21 = cabs1(H[(long)(M + 1) * m + M]);
            const double sc = a11 + a21;                      // > 0: H[M+1][M] did not deflate
            const double h10 = cabs1(H[(long)M * m + M - 1]);
            if (h10 * (a21 / sc) <= ulp * ((a11 / sc) * (cabs1(h11) + cabs1(h22)))) atomicMax(&lst, M);
        }
        __syncthreads();
        const int ks = lst;
        for (int k = ks; k < ihi; ++k) {
            zd x, y;
            if (k == ks) { x = H[(long)ks * m + ks] - mu; y = H[(long)(ks + 1) * m + ks]; }
            else { x = H[(long)k * m + k - 1]; y = H[(long)(k + 1) * m + k - 1]; }
            double c; zd s, r;
            givens(x, y, c, s, r);
            __syncthreads();
            const int j0 = (k == ks) ? ks : k - 1;
            for (int j = j0 + tid; j < m; j += ENT) {
                const zd h1 = H[(long)k * m + j], h2 = H[(long)(k + 1) * m + j];
                zd n1 = c * h1; cfma(n1, s, h2);
                zd n2 = c * h2; cfms(n2, conj(s), h1);
                H[(long)k * m + j] = n1;
                H[(long)(k + 1) * m + j] = n2;
            }
            __syncthreads();
            if (tid == 0) {
                if (k > ks) { H[(long)k * m + k - 1] = r; H[(long)(k + 1) * m + k - 1] = czero<double>(); }
                else if (ks > l) H[(long)ks * m + ks - 1] = c * H[(long)ks * m + ks - 1];   // fill-in below: dropped
            }
            const int iend = min(k + 2, ihi);
            for (int i = tid; i < (iend + 1) + m; i += ENT) {
                zd* R = (i <= iend) ? (H + (long)i * m) : (Z + (long)(i - iend - 1) * m);
                const zd h1 = R[k], h2 = R[k + 1];
                zd n1 = c * h1; cfma(n1, conj(s), h2);
                zd n2 = c * h2; cfms(n2, s, h1);
                R[k] = n1;
                R[k + 1] = n2;
            }
            __syncthreads();
        }
        if (++its > 30 * max(10, m)) return 1;   // per deflation, as LAPACK's ITMAX
    }
    __syncthreads();
    return 0;
}

// V = Z X with X the eigenvectors of the triangular T; unit 2-norm columns
__device__ void schur_vectors(int m, const zd* T, const zd* Z, zd* X, zd* V, double* red) {
    const int tid = threadIdx.x;
    const double ulp = DBL_EPSILON, smlnum = DBL_MIN * (double(m) / DBL_EPSILON);
    for (int k = tid; k < m; k += ENT) {
        const zd tkk = T[(long)k * m + k];
        const double smin = fmax(ulp * cabs1(tkk), smlnum);
        for (int i = k + 1; i < m; ++i) X[(long)i * m + k] = czero<double>();
        X[(long)k * m + k] = cx(1.0, 0.0);
        for (int i = k - 1; i >= 0; --i) {
            zd s = T[(long)i * m + k];
            for (int j = i + 1; j < k; ++j) cfma(s, T[(long)i * m + j], X[(long)j * m + k]);
            zd d = T[(long)i * m + i] - tkk;
            if (cabs1(d) < smin) d = cx(smin, 0.0);
            X[(long)i * m + k] = -cdiv(s, d);
        }
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += ENT) {
        const int i = e / m, k = e % m;
        zd s = czero<double>();
        for (int j = 0; j <= k; ++j) cfma(s, Z[(long)i * m + j], X[(long)j * m + k]);
        V[e] = s;
    }
    __syncthreads();
    for (int k = tid; k < m; k += ENT) {
        double nn = 0.0;
        for (int i = 0; i < m; ++i) nn += abs2(V[(long)i * m + k]);
        const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 1.0;
        for (int i = 0; i < m; ++i) V[(long)i * m + k] = inv * V[(long)i * m + k];
    }
    __syncthreads();
}

// Gauss-Jordan with partial pivoting on Aug (m x w, ld w): [A | R] -> [I | A^{-1} R]
__device__ int gauss_jordan(int m, int w, zd* Aug, zd* f, double* red, int* redi) {
    const int tid = threadIdx.x;
    int bad = 0;
    for (int k = 0; k < m; ++k) {
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < m; i += ENT) {
            double v = cabs1(Aug[(long)i * w + k]);
            if (v > best) { best = v; bi = i; }
        }
        red[tid] = best;
        redi[tid] = bi;
        __syncthreads();
        for (int s = ENT / 2; s > 0; s >>= 1) {
            if (tid < s) {
                if (red[tid + s] > red[tid] || (red[tid + s] == red[tid] && redi[tid + s] < redi[tid])) {
                    red[tid] = red[tid + s];
                    redi[tid] = redi[tid + s];
                }
            }
            __syncthreads();
        }
        const int p = redi[0];
        if (!(red[0] > 0.0)) bad = 1;
        __syncthreads();
        if (p != k)
            for (int j = tid; j < w; j += ENT) {
                zd t = Aug[(long)k * w + j];
                Aug[(long)k * w + j] = Aug[(long)p * w + j];
                Aug[(long)p * w + j] = t;
            }
        __syncthreads();
        const zd inv = bad ? cx(1.0, 0.0) : cdiv(cx(1.0, 0.0), Aug[(long)k * w + k]);
        __syncthreads();
        for (int j = tid; j < w; j += ENT) Aug[(long)k * w + j] = Aug[(long)k * w + j] * inv;
        for (int i = tid; i < m; i += ENT) f[i] = (i == k) ? czero<double>() : Aug[(long)i * w + k];
        __syncthreads();
        for (int e = tid; e < m * w; e += ENT) {
            const int i = e / w, j = e % w;
            if (i != k) cfms(Aug[e], f[i], Aug[(long)k * w + j]);
        }
        __syncthreads();
    }
    return bad;
}

// Work layout (complex): H, Z, X, V, Vi (m*m each), Aug (m*3m), v, f (m each)
static size_t eig_work_elems(int m) { return (size_t)m * m * 8 + 2 * (size_t)m + 64; }

// H and Z of the reduction and the QR iteration live in LDS when m <= 64
// (dynamic shared memory of 2 m^2 entries): every one of the QR iteration's
// dependent Givens steps then waits on LDS, not on global memory.
constexpr int EIG_LDS_M = 64;

__device__ void eig_core(int m, zd* H, zd* Z, zd* X, zd* V, zd* v, double* red, int* info, bool loose) {
    const int tid = threadIdx.x;
    extern __shared__ unsigned char eig_dsm[];
    const bool lds = m <= EIG_LDS_M;
    zd* Hw = lds ? (zd*)eig_dsm : H;
    zd* Zw = lds ? (zd*)eig_dsm + (size_t)m * m : Z;
    for (int e = tid; e < m * m; e += ENT) {
        Zw[e] = (e / m == e % m) ? cx(1.0, 0.0) : czero<double>();
        if (lds) Hw[e] = H[e];
    }
    __syncthreads();
    hessenberg(m, Hw, Zw, v, red);
    int bad = schur_qr(m, Hw, Zw, loose);
    if (lds) {
        for (int e = tid; e < m * m; e += ENT) {
            H[e] = Hw[e];
            Z[e] = Zw[e];
        }
        __syncthreads();
    }
    if (bad && tid == 0) *info = 1;
    schur_vectors(m, H, Z, X, V, red);
}

__device__ void biortho_body(int m, const zd* __restrict__ BQ, double eta, zd* __restrict__ gamma,
                             zd* __restrict__ S, zd* __restrict__ Sh, int* __restrict__ m0t, int* __restrict__ info,
                             zd* __restrict__ work, double* red, int* redi, int* sorder) {
    const int tid = threadIdx.x;
    const size_t mm = (size_t)m * m;
    zd *H = work, *Z = H + mm, *X = Z + mm, *V = X + mm, *Aug = V + mm, *v = Aug + 3 * mm, *f = v + m;
    if (tid == 0) *info = 0;
    for (size_t e = tid; e < mm; e += ENT) H[e] = BQ[e];
    __syncthreads();
    eig_core(m, H, Z, X, V, v, red, info, true);
    // gamma (unsorted) = diag(T)
    // V^{-1} by Gauss-Jordan on [V | I]
    for (int e = tid; e < 2 * m * m; e += ENT) {
        const int i = e / (2 * m), j = e % (2 * m);
        Aug[e] = (j < m) ? V[(long)i * m + j] : ((j - m == i) ? cx(1.0, 0.0) : czero<double>());
    }
    __syncthreads();
    int bad = gauss_jordan(m, 2 * m, Aug, f, red, redi);
    if (bad && tid == 0) *info = 2;
    // stable descending sort of |gamma|
    for (int i = tid; i < m; i += ENT) {
        const double gi = cabs(H[(long)i * m + i]);
        int r = 0;
        for (int j = 0; j < m; ++j) {
            const double gj = cabs(H[(long)j * m + j]);
            if (gj > gi || (gj == gi && j < i)) ++r;
        }
        sorder[r] = i;
        if (!(gi == gi) && tid == 0) *info = 3;
    }
    __syncthreads();
    double gmax = 0.0;
    for (int i = 0; i < m; ++i) gmax = fmax(gmax, cabs(H[(long)i * m + i]));
    int cnt = 0;
    for (int i = 0; i < m; ++i) cnt += (cabs(H[(long)i * m + i]) >= eta * gmax) ? 1 : 0;
    if (tid == 0) *m0t = cnt;
    for (int r = tid; r < m; r += ENT) gamma[r] = H[(long)sorder[r] * m + sorder[r]];
    // S[:, r] = V[:, o] g^{-1/2};  Sh[:, r] = Vh[:, o] conj(g^{-1/2}), Vh[i][o] = conj(Vinv[o][i])
    for (int e = tid; e < m * m; e += ENT) {
        const int i = e / m, r = e % m;
        if (r < cnt) {
            const int o = sorder[r];
            const zd g = H[(long)o * m + o];
            const zd s = cdiv(cx(1.0, 0.0), csqrt(g));
            S[e] = V[(long)i * m + o] * s;
            Sh[e] = conj(Aug[(long)o * 2 * m + m + i]) * conj(s);
        } else {
            S[e] = czero<double>();
            Sh[e] = czero<double>();
        }
    }
}

__device__ void reduced_body(int m, const zd* __restrict__ AU, const zd* __restrict__ BU, zd* __restrict__ lam,
                             zd* __restrict__ W, zd* __restrict__ Wh, int* __restrict__ info, zd* __restrict__ work,
                             double* red, int* redi) {
    const int tid = threadIdx.x;
    const size_t mm = (size_t)m * m;
    zd *H = work, *Z = H + mm, *X = Z + mm, *V = X + mm, *Aug = V + mm, *v = Aug + 3 * mm, *f = v + m;
    if (tid == 0) *info = 0;
    // [B_U | A_U | I] -> [I | B_U^{-1} A_U | B_U^{-1}]
    const int w3 = 3 * m;
    for (int e = tid; e < m * w3; e += ENT) {
        const int i = e / w3, j = e % w3;
        zd val;
        if (j < m) val = BU[(long)i * m + j];
        else if (j < 2 * m) val = AU[(long)i * m + j - m];
        else val = (j - 2 * m == i) ? cx(1.0, 0.0) : czero<double>();
        Aug[e] = val;
    }
    __syncthreads();
    int bad = gauss_jordan(m, w3, Aug, f, red, redi);
    if (bad && tid == 0) *info = 2;
    for (int e = tid; e < (int)mm; e += ENT) H[e] = Aug[(long)(e / m) * w3 + m + (e % m)];
    __syncthreads();
    eig_core(m, H, Z, X, V, v, red, info, false);
    for (int i = tid; i < m; i += ENT) lam[i] = H[(long)i * m + i];
    for (size_t e = tid; e < mm; e += ENT) W[e] = V[e];
    // keep B_U^{-1} (right third of Aug) in X
    for (int e = tid; e < (int)mm; e += ENT) X[e] = Aug[(long)(e / m) * w3 + 2 * m + (e % m)];
    __syncthreads();
    // W^{-1} by Gauss-Jordan on [V | I] (reuse Aug with width 2m)
    for (int e = tid; e < 2 * m * m; e += ENT) {
        const int i = e / (2 * m), j = e % (2 * m);
        Aug[e] = (j < m) ? V[(long)i * m + j] : ((j - m == i) ? cx(1.0, 0.0) : czero<double>());
    }
    __syncthreads();
    bad = gauss_jordan(m, 2 * m, Aug, f, red, redi);
    if (bad && tid == 0) *info = 2;
    // Wh^H = W^{-1} B_U^{-1}  ->  Wh[i][k] = conj( (W^{-1} B_U^{-1})[k][i] )
    for (int e = tid; e < (int)mm; e += ENT) {
        const int k = e / m, i = e % m;
        zd s = czero<double>();
        for (int j = 0; j < m; ++j) cfma(s, Aug[(long)k * 2 * m + m + j], X[(long)j * m + i]);
        Wh[(long)i * m + k] = conj(s);
    }
}

__global__ __launch_bounds__(ENT) void k_eig_biortho(int m, const zd* __restrict__ BQ, double eta, zd* __restrict__ gamma,
                                                     zd* __restrict__ S, zd* __restrict__ Sh, int* __restrict__ m0t,
                                                     int* __restrict__ info, zd* __restrict__ work) {
    __shared__ double red[ENT];
    __shared__ int redi[ENT];
    __shared__ int sorder[1024];
    biortho_body(m, BQ, eta, gamma, S, Sh, m0t, info, work, red, redi, sorder);
}

__global__ __launch_bounds__(ENT) void k_eig_reduced(int m, const zd* __restrict__ AU, const zd* __restrict__ BU,
                                                     zd* __restrict__ lam, zd* __restrict__ W, zd* __restrict__ Wh,
                                                     int* __restrict__ info, zd* __restrict__ work) {
    __shared__ double red[ENT];
    __shared__ int redi[ENT];
    reduced_body(m, AU, BU, lam, W, Wh, info, work, red, redi);
}

// batched: one workgroup per problem of the list
__global__ __launch_bounds__(ENT) void k_eig_biortho_b(const EigJob* __restrict__ jobs) {
    __shared__ double red[ENT];
    __shared__ int redi[ENT];
    __shared__ int sorder[1024];
    const EigJob j = jobs[blockIdx.x];
    biortho_body(j.m, j.in1, j.eta, j.out0, j.out1, j.out2, j.i0, j.i1, j.work, red, redi, sorder);
}

__global__ __launch_bounds__(ENT) void k_eig_reduced_b(const EigJob* __restrict__ jobs) {
    __shared__ double red[ENT];
    __shared__ int redi[ENT];
    const EigJob j = jobs[blockIdx.x];
    reduced_body(j.m, j.in1, j.in2, j.out0, j.out1, j.out2, j.i0, j.work, red, redi);
}

size_t eig_work_size(int m) { return sizeof(zd) * eig_work_elems(m); }

// dynamic LDS of the eigensolver kernels for problems up to size mmax
static size_t eig_lds_bytes(int mmax) {
    static bool attr = false;
    if (!attr) {
        const int b = (int)(2 * sizeof(zd) * EIG_LDS_M * EIG_LDS_M);   // 128 KiB of the 160 KiB per workgroup
        FH_HIP(hipFuncSetAttribute((const void*)k_eig_biortho, hipFuncAttributeMaxDynamicSharedMemorySize, b));
        FH_HIP(hipFuncSetAttribute((const void*)k_eig_reduced, hipFuncAttributeMaxDynamicSharedMemorySize, b));
        FH_HIP(hipFuncSetAttribute((const void*)k_eig_biortho_b, hipFuncAttributeMaxDynamicSharedMemorySize, b));
        FH_HIP(hipFuncSetAttribute((const void*)k_eig_reduced_b, hipFuncAttributeMaxDynamicSharedMemorySize, b));
        attr = true;
    }
    const int mm = std::min(mmax, EIG_LDS_M);
    return 2 * sizeof(zd) * (size_t)mm * mm;
}

void eig_biortho(hipStream_t st, int m, const zd* BQ, double eta, zd* gamma, zd* S, zd* Sh, int* m0t, int* info,
                 DBuf& work) {
    FH_REQUIRE(m >= 1 && m <= 1024, -2, "eig_biortho: m out of range");
    zd* w = (zd*)work.ensure(sizeof(zd) * eig_work_elems(m));
    k_eig_biortho<<<1, ENT, eig_lds_bytes(m), st>>>(m, BQ, eta, gamma, S, Sh, m0t, info, w);
    FH_LAUNCH_CHECK();
}
void eig_reduced(hipStream_t st, int m, const zd* AU, const zd* BU, zd* lam, zd* W, zd* Wh, int* info, DBuf& work) {
    FH_REQUIRE(m >= 1 && m <= 1024, -2, "eig_reduced: m out of range");
    zd* w = (zd*)work.ensure(sizeof(zd) * eig_work_elems(m));
    k_eig_reduced<<<1, ENT, eig_lds_bytes(m), st>>>(m, AU, BU, lam, W, Wh, info, w);
    FH_LAUNCH_CHECK();
}
void eig_biortho_batched(hipStream_t st, int count, const EigJob* jobs_dev, int mmax) {
    if (count <= 0) return;
    k_eig_biortho_b<<<count, ENT, eig_lds_bytes(mmax), st>>>(jobs_dev);
    FH_LAUNCH_CHECK();
}
void eig_reduced_batched(hipStream_t st, int count, const EigJob* jobs_dev, int mmax) {
    if (count <= 0) return;
    k_eig_reduced_b<<<count, ENT, eig_lds_bytes(mmax), st>>>(jobs_dev);
    FH_LAUNCH_CHECK();
}

}  // namespace fh
