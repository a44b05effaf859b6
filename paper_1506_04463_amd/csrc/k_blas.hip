// Dense complex kernels: tiled GEMM (row-major, conjugate-transpose
// operands), tall-skinny reductions X^H Y, eq:res column norms, contour
// accumulation, copies and casts.
#include "fh_kernels.h"

namespace fh {

// ---------------------------------------------------------------------------
// GEMM: 64x64 output tile per workgroup, K in steps of 16 staged through LDS;
// each of the 256 threads owns a 4x4 complex micro-tile (rows ty+16a,
// cols tx+16b).  kchunk > 0 splits K across the batch index (split-K).
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;

template <typename T, bool AH, bool BH>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, Cx<T> alpha, const Cx<T>* __restrict__ A,
                                              long lda, long sA, const Cx<T>* __restrict__ B, long ldb, long sB,
                                              Cx<T> beta, Cx<T>* __restrict__ C, long ldc, long sC, int kchunk) {
    const int bz = blockIdx.z;
    A += bz * sA;
    B += bz * sB;
    C += bz * sC;
    int Keff = K;
    if (kchunk > 0) Keff = min(kchunk, K - bz * kchunk);
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    __shared__ Cx<T> As[GK][GT + 1];
    __shared__ Cx<T> Bs[GK][GT + 1];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    Cx<T> acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = czero<T>();

    for (int k0 = 0; k0 < Keff; k0 += GK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int e = tid + 256 * q;
            int i, kk;
            if (!AH) { i = e / GK; kk = e % GK; } else { kk = e / GT; i = e % GT; }
            int gi = m0 + i, gk = k0 + kk;
            Cx<T> v = czero<T>();
            if (gi < M && gk < Keff) v = AH ? conj(A[(long)gk * lda + gi]) : A[(long)gi * lda + gk];
            As[kk][i] = v;
            int j;
            if (!BH) { kk = e / GT; j = e % GT; } else { j = e / GK; kk = e % GK; }
            int gj = n0 + j;
            gk = k0 + kk;
            Cx<T> u = czero<T>();
            if (gj < N && gk < Keff) u = BH ? conj(B[(long)gj * ldb + gk]) : B[(long)gk * ldb + gj];
            Bs[kk][j] = u;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            Cx<T> av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < 4; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) cfma(acc[a][b], av[a], bv[b]);
        }
        __syncthreads();
    }
    const bool use_beta = (beta.re != T(0) || beta.im != T(0));
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        int gi = m0 + ty + 16 * a;
        if (gi >= M) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int gj = n0 + tx + 16 * b;
            if (gj >= N) continue;
            Cx<T> r = alpha * acc[a][b];
            if (use_beta) cfma(r, beta, C[(long)gi * ldc + gj]);
            C[(long)gi * ldc + gj] = r;
        }
    }
}

template <typename T>
void gemm(hipStream_t st, char opA, char opB, int M, int N, int K, Cx<T> alpha, const Cx<T>* A, long lda,
          long sA, const Cx<T>* B, long ldb, long sB, Cx<T> beta, Cx<T>* C, long ldc, long sC, int batch) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    dim3 grid(ceil_div(N, GT), ceil_div(M, GT), batch);
    const bool ah = (opA == 'C'), bh = (opB == 'C');
    if (!ah && !bh) k_gemm<T, false, false><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 0);
    else if (ah && !bh) k_gemm<T, true, false><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 0);
    else if (!ah && bh) k_gemm<T, false, true><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 0);
    else k_gemm<T, true, true><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, 0);
    FH_LAUNCH_CHECK();
}
template void gemm<double>(hipStream_t, char, char, int, int, int, zd, const zd*, long, long, const zd*, long,
                           long, zd, zd*, long, long, int);
template void gemm<float>(hipStream_t, char, char, int, int, int, cf, const cf*, long, long, const cf*, long,
                          long, cf, cf*, long, long, int);

// sum of `parts` partial p x q blocks (stride p*q) into C (ld), fixed order
__global__ void k_reduce_parts(int parts, int p, int q, const zd* __restrict__ P, zd* __restrict__ C, long ldc) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= p * q) return;
    zd s = czero<double>();
    for (int b = 0; b < parts; ++b) s = s + P[(long)b * p * q + e];
    C[(long)(e / q) * ldc + (e % q)] = s;
}

// split of the n rows into `parts` chunks of `chunk` rows (multiple of 16 when
// coarsened) with at most max_parts parts
static void tall_split(int n, int max_parts, int& chunk, int& parts) {
    chunk = 256;
    parts = ceil_div(n, chunk);
    if (parts > max_parts) {
        chunk = ceil_div(n, max_parts);
        chunk = (chunk + 15) / 16 * 16;
        parts = ceil_div(n, chunk);
    }
}

static void tall_launch(hipStream_t st, int n, int p, int q, const zd* X, long ldx, const zd* Y, long ldy, zd* C,
                        long ldc, zd* P, int chunk, int parts) {
    dim3 grid(ceil_div(q, GT), ceil_div(p, GT), parts);
    k_gemm<double, true, false><<<grid, 256, 0, st>>>(p, q, n, cx(1.0, 0.0), X, ldx, (long)chunk * ldx, Y, ldy,
                                                       (long)chunk * ldy, czero<double>(), P, q, (long)p * q, chunk);
    FH_LAUNCH_CHECK();
    k_reduce_parts<<<ceil_div((size_t)p * q, 256), 256, 0, st>>>(parts, p, q, P, C, ldc);
    FH_LAUNCH_CHECK();
}

bool gemm_hn_tall_into(hipStream_t st, int n, int p, int q, const zd* X, long ldx, const zd* Y, long ldy, zd* C,
                       long ldc, void* part, size_t cap) {
    if (p <= 0 || q <= 0) return true;
    const size_t per = sizeof(zd) * (size_t)p * q;
    const size_t fit = cap / per;
    if (fit < 1) return false;
    int chunk, parts;
    tall_split(n, (int)std::min<size_t>(fit, 1024), chunk, parts);
    tall_launch(st, n, p, q, X, ldx, Y, ldy, C, ldc, (zd*)part, chunk, parts);
    return true;
}

void gemm_hn_tall(hipStream_t st, int n, int p, int q, const zd* X, long ldx, const zd* Y, long ldy, zd* C,
                  long ldc, DBuf& partial) {
    if (p <= 0 || q <= 0) return;
    int chunk, parts;
    tall_split(n, 1024, chunk, parts);
    zd* P = (zd*)partial.ensure(sizeof(zd) * (size_t)parts * p * q);
    tall_launch(st, n, p, q, X, ldx, Y, ldy, C, ldc, P, chunk, parts);
}

// ---------------------------------------------------------------------------
// eq:res column norms: block (m, ry); partials per row chunk then reduction
// ---------------------------------------------------------------------------
__global__ void k_res_partial(int n, int m, const zd* __restrict__ AY, const zd* __restrict__ BY, long ld,
                              const zd* __restrict__ lam, int conj_lam, int rows_per_chunk, double* __restrict__ part) {
    extern __shared__ double sh[];
    const int c = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const int r0 = blockIdx.x * rows_per_chunk, r1 = min(n, r0 + rows_per_chunk);
    zd l = lam[c];
    if (conj_lam) l = conj(l);
    double num = 0.0, den = 0.0;
    for (int r = r0 + ty; r < r1; r += ry) {
        zd b = BY[(long)r * ld + c];
        zd d = AY[(long)r * ld + c];
        cfms(d, l, b);
        num += cabs(d);
        den += cabs(b);
    }
    double* sn = sh;
    double* sd = sh + ry * m;
    sn[ty * m + c] = num;
    sd[ty * m + c] = den;
    __syncthreads();
    if (ty == 0) {
        for (int t = 1; t < ry; ++t) { num += sn[t * m + c]; den += sd[t * m + c]; }
        part[(long)blockIdx.x * 2 * m + c] = num;
        part[(long)blockIdx.x * 2 * m + m + c] = den;
    }
}

__global__ void k_res_reduce(int parts, int m, const double* __restrict__ part, double* num, double* den) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    double a = 0.0, b = 0.0;
    for (int p = 0; p < parts; ++p) { a += part[(long)p * 2 * m + c]; b += part[(long)p * 2 * m + m + c]; }
    num[c] = a;
    den[c] = b;
}

void res_colnorms(hipStream_t st, int n, int m, const zd* AY, const zd* BY, long ld, const zd* lam, bool conj_lam,
                  double* num, double* den, DBuf& partial) {
    if (m <= 0) return;
    int ry = m >= 256 ? 1 : 256 / m;
    int rows = 512;
    int parts = ceil_div(n, rows);
    double* P = (double*)partial.ensure(sizeof(double) * 2 * (size_t)parts * m);
    dim3 blk(m, ry);
    k_res_partial<<<parts, blk, 2 * sizeof(double) * ry * m, st>>>(n, m, AY, BY, ld, lam, conj_lam ? 1 : 0, rows, P);
    FH_LAUNCH_CHECK();
    k_res_reduce<<<ceil_div(m, 128), 128, 0, st>>>(parts, m, P, num, den);
    FH_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// contour accumulation Q = sum_j c_j X_j (summation order j = 0..ne-1)
// ---------------------------------------------------------------------------
__global__ void k_accumulate(int ne, long len, const zd* __restrict__ X, long sX, const zd* __restrict__ w,
                             int conj_w, zd* __restrict__ Q) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    zd s = czero<double>();
    for (int j = 0; j < ne; ++j) {
        zd c = w[j];
        if (conj_w) c = conj(c);
        cfma(s, c, X[(long)j * sX + e]);
    }
    Q[e] = s;
}

void accumulate(hipStream_t st, int ne, long len, const zd* X, long strideX, const zd* w_dev, bool conj_w, zd* Q) {
    if (len <= 0) return;
    k_accumulate<<<ceil_div(len, 256), 256, 0, st>>>(ne, len, X, strideX, w_dev, conj_w ? 1 : 0, Q);
    FH_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_replicate(long len, const Cx<T>* __restrict__ src, Cx<T>* __restrict__ dst, int copies) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    Cx<T> v = src[e];
    for (int j = 0; j < copies; ++j) dst[(long)j * len + e] = v;
}
template <typename T>
void replicate(hipStream_t st, long len, const Cx<T>* src, Cx<T>* dst, int copies) {
    if (len <= 0 || copies <= 0) return;
    k_replicate<T><<<ceil_div(len, 256), 256, 0, st>>>(len, src, dst, copies);
    FH_LAUNCH_CHECK();
}
template void replicate<double>(hipStream_t, long, const zd*, zd*, int);
template void replicate<float>(hipStream_t, long, const cf*, cf*, int);

// dst = conj(src), elementwise
__global__ void k_conj_copy(long len, const zd* __restrict__ src, zd* __restrict__ dst) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    const zd v = src[e];
    dst[e] = zd{v.re, -v.im};
}
void conj_copy(hipStream_t st, long len, const zd* src, zd* dst) {
    if (len <= 0) return;
    k_conj_copy<<<ceil_div(len, 256), 256, 0, st>>>(len, src, dst);
    FH_LAUNCH_CHECK();
}

// Left block of a complex symmetric filter: Qh = conj(Q) D with
// D = diag(conj(1 / s_c)), s_c = sum_r Y[r][c]^2 (bilinear, no conjugate).
// Partial sums of s per chunk of rows, one thread per column
__global__ void k_bilin_partial(int n, int m, const zd* __restrict__ Y, int rows, zd* __restrict__ part) {
    const int c = threadIdx.x, ch = blockIdx.x;
    if (c >= m) return;
    const int r0 = ch * rows, r1 = min(n, r0 + rows);
    zd s = czero<double>();
    for (int r = r0; r < r1; ++r) {
        const zd y = Y[(long)r * m + c];
        cfma(s, y, y);
    }
    part[(long)ch * m + c] = s;
}
__global__ void k_bilin_scale(int nch, int m, const zd* __restrict__ part, const zd* __restrict__ Y0, zd* __restrict__ d) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    zd s = czero<double>();
    for (int ch = 0; ch < nch; ++ch) s = s + part[(long)ch * m + c];
    const double a = cabs(s);
    // a quasi-null column (y^T y = 0) keeps the plain conjugate
    d[c] = (a > 0.0 && std::isfinite(a)) ? conj(cdiv(cx(1.0, 0.0), s)) : cx(1.0, 0.0);
}
__global__ void k_conj_copy_cols(long len, int m, const zd* __restrict__ src, const zd* __restrict__ d,
                                 zd* __restrict__ dst) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    dst[e] = conj(src[e]) * d[e % m];
}
void conj_copy_bilin(hipStream_t st, int n, int m, const zd* Y, const zd* Q, zd* Qh, DBuf& part) {
    if (n <= 0 || m <= 0) return;
    const int rows = 256, nch = ceil_div(n, rows);
    zd* P = (zd*)part.ensure(sizeof(zd) * ((size_t)nch * m + m));
    zd* d = P + (size_t)nch * m;
    k_bilin_partial<<<nch, ((m + 63) / 64) * 64, 0, st>>>(n, m, Y, rows, P);
    FH_LAUNCH_CHECK();
    k_bilin_scale<<<ceil_div(m, 64), 64, 0, st>>>(nch, m, P, Y, d);
    FH_LAUNCH_CHECK();
    const long len = (long)n * m;
    k_conj_copy_cols<<<ceil_div(len, 256), 256, 0, st>>>(len, m, Q, d, Qh);
    FH_LAUNCH_CHECK();
}

// Conjugation-closed columns, in place.  cp is an involution on the m
// columns: a pair (i, k = cp[i] > i) gets x_k = conj(x_i); a column with
// cp[c] = c is made real as Re(x_c e^{-i phi_c / 2}), phi_c = arg(x_c^T x_c):
// for x_c = e^{i t} r with r real, x_c^T x_c = e^{2 i t} r^T r, so the product
// is +-r (the real eigenvector of a real eigenvalue, up to its sign).  A
// second block (the left vectors, xh_c^H x_c = 1) takes the same operations
// with the phases of the first, which keeps xh_c^H x_c = 1.
__global__ void k_conj_phase(int nch, int m, const zd* __restrict__ part, const int* __restrict__ cp,
                             zd* __restrict__ ph) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    zd s = czero<double>();
    for (int ch = 0; ch < nch; ++ch) s = s + part[(long)ch * m + c];
    zd p = cx(1.0, 0.0);
    if (cp[c] == c && cabs(s) > 0.0 && std::isfinite(cabs(s))) {
        const double h = 0.5 * atan2(s.im, s.re);
        p = cx(cos(h), -sin(h));
    }
    ph[c] = p;
}
__global__ void k_conj_close(long len, int m, const int* __restrict__ cp, const zd* __restrict__ ph,
                             zd* __restrict__ X) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    const int c = e % m, pc = cp[c];
    if (pc == c) {
        const zd v = X[e] * ph[c];
        X[e] = cx(v.re, 0.0);
    } else if (pc < c) {
        X[e] = conj(X[e - c + pc]);
    }
}
void conj_close_cols(hipStream_t st, int n, int m, zd* X, zd* Xh, const int* cp_dev, DBuf& part) {
    if (n <= 0 || m <= 0) return;
    const int rows = 256, nch = ceil_div(n, rows);
    zd* P = (zd*)part.ensure(sizeof(zd) * ((size_t)nch * m + m));
    zd* ph = P + (size_t)nch * m;
    k_bilin_partial<<<nch, ((m + 63) / 64) * 64, 0, st>>>(n, m, X, rows, P);
    FH_LAUNCH_CHECK();
    k_conj_phase<<<ceil_div(m, 64), 64, 0, st>>>(nch, m, P, cp_dev, ph);
    FH_LAUNCH_CHECK();
    const long len = (long)n * m;
    k_conj_close<<<ceil_div(len, 256), 256, 0, st>>>(len, m, cp_dev, ph, X);
    FH_LAUNCH_CHECK();
    if (Xh) {
        k_conj_close<<<ceil_div(len, 256), 256, 0, st>>>(len, m, cp_dev, ph, Xh);
        FH_LAUNCH_CHECK();
    }
}

// X = Re(X) in place
__global__ void k_real_part(long len, zd* __restrict__ X) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) X[e].im = 0.0;
}
void real_part(hipStream_t st, long len, zd* X) {
    if (len <= 0) return;
    k_real_part<<<ceil_div(len, 256), 256, 0, st>>>(len, X);
    FH_LAUNCH_CHECK();
}

template <typename D, typename S>
__global__ void k_cast(long len, const Cx<S>* __restrict__ src, Cx<D>* __restrict__ dst) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) dst[e] = ccast<D>(src[e]);
}
template <typename D, typename S>
void cast(hipStream_t st, long len, const Cx<S>* src, Cx<D>* dst) {
    if (len <= 0) return;
    k_cast<D, S><<<ceil_div(len, 256), 256, 0, st>>>(len, src, dst);
    FH_LAUNCH_CHECK();
}
template void cast<float, double>(hipStream_t, long, const zd*, cf*);
template void cast<double, float>(hipStream_t, long, const cf*, zd*);

__global__ void k_shift_combine(long len, zd s, const zd* __restrict__ X, zd* __restrict__ Out) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    zd o = -Out[e];
    cfma(o, s, X[e]);
    Out[e] = o;
}
void shift_combine(hipStream_t st, long len, zd s, const zd* X, zd* Out) {
    if (len <= 0) return;
    k_shift_combine<<<ceil_div(len, 256), 256, 0, st>>>(len, s, X, Out);
    FH_LAUNCH_CHECK();
}

__global__ void k_sub(long len, const zd* __restrict__ A, const zd* __restrict__ B, zd* __restrict__ Out) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) Out[e] = A[e] - B[e];
}
void sub(hipStream_t st, long len, const zd* A, const zd* B, zd* Out) {
    if (len <= 0) return;
    k_sub<<<ceil_div(len, 256), 256, 0, st>>>(len, A, B, Out);
    FH_LAUNCH_CHECK();
}

__global__ void k_gather_cols(int n, int mout, const zd* __restrict__ src, long lds, const int* __restrict__ perm,
                              zd* __restrict__ dst, long ldd) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * mout) return;
    int i = e / mout, k = e % mout;
    dst[(long)i * ldd + k] = src[(long)i * lds + perm[k]];
}
void gather_cols(hipStream_t st, int n, int mout, const zd* src, long lds, const int* perm_dev, zd* dst, long ldd) {
    if (n <= 0 || mout <= 0) return;
    k_gather_cols<<<ceil_div((size_t)n * mout, 256), 256, 0, st>>>(n, mout, src, lds, perm_dev, dst, ldd);
    FH_LAUNCH_CHECK();
}

}  // namespace fh
