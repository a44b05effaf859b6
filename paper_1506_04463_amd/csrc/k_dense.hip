// Dense shifted systems of the contour filter (Section 2.4: one LU of
// (z_j B - A) per node, reused for the right solve and, through a
// conjugate-transpose solve, for the left solve).
//
// Row-major storage.  LU with partial pivoting, right-looking and blocked:
// panel factorization (one workgroup per matrix), triangular solve of the
// U12 block row, and a trailing rank-nb update by the tiled GEMM.  Solves are
// blocked the same way: diagonal-block triangular solves in LDS plus GEMM
// updates of the remaining rows.
#include "fh_kernels.h"

namespace fh {

constexpr int NB = 32;   // panel / block width

__global__ void k_form_shift(int n, const zd* __restrict__ A, long lda, const zd* __restrict__ B, long ldb,
                             const zd* __restrict__ z, zd* __restrict__ M) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (e >= (long)n * n) return;
    int r = e / n, c = e % n;
    zd zj = z[j];
    zd v = -A[(long)r * lda + c];
    if (B) cfma(v, zj, B[(long)r * ldb + c]);
    else if (r == c) v = v + zj;
    M[(long)j * n * n + e] = v;
}

void form_shift(hipStream_t st, int n, const zd* A, long lda, const zd* B, long ldb, int ne, const zd* z_dev, zd* M) {
    dim3 grid(ceil_div((size_t)n * n, 256), ne);
    k_form_shift<<<grid, 256, 0, st>>>(n, A, lda, B, ldb, z_dev, M);
    FH_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// panel: columns [k, k+jb) of rows [k, n); pivot search by |re|+|im| with
// the lowest index on ties; row interchanges applied to the full row.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(NT) void k_lu_panel(int n, zd* __restrict__ Mall, int k, int jb, int* __restrict__ ipiv,
                                                 int* __restrict__ info) {
    zd* A = Mall + (long)blockIdx.x * n * n;
    int* piv = ipiv + (long)blockIdx.x * n;
    const long ld = n;
    __shared__ double sv[NT];
    __shared__ int si[NT];
    const int tid = threadIdx.x;
    for (int c = k; c < k + jb; ++c) {
        double best = -1.0;
        int bi = c;
        for (int i = c + tid; i < n; i += NT) {
            double v = cabs1(A[(long)i * ld + c]);
            if (v > best) { best = v; bi = i; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (tid < s) {
                double o = sv[tid + s];
                int oi = si[tid + s];
                if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
            }
            __syncthreads();
        }
        const int p = si[0];
        const double pv = sv[0];
        __syncthreads();
        if (tid == 0) {
            piv[c] = p;
            if (!(pv > 0.0) && info[blockIdx.x] == 0) info[blockIdx.x] = c + 1;
        }
        if (p != c) {
            for (int j = tid; j < n; j += NT) {
                zd t = A[(long)c * ld + j];
                A[(long)c * ld + j] = A[(long)p * ld + j];
                A[(long)p * ld + j] = t;
            }
        }
        __syncthreads();
        if (pv > 0.0) {
            const zd dinv = cdiv(cx(1.0, 0.0), A[(long)c * ld + c]);
            for (int i = c + 1 + tid; i < n; i += NT) {
                zd l = A[(long)i * ld + c] * dinv;
                A[(long)i * ld + c] = l;
                for (int j = c + 1; j < k + jb; ++j) cfms(A[(long)i * ld + j], l, A[(long)c * ld + j]);
            }
        }
        __syncthreads();
    }
}

// U12 = L11^{-1} A12 for rows [k, k+jb), columns [k+jb, n) in 64-wide tiles
__global__ __launch_bounds__(256) void k_lu_trsm_row(int n, zd* __restrict__ Mall, int k, int jb) {
    zd* A = Mall + (long)blockIdx.y * n * n;
    const long ld = n;
    __shared__ zd L[NB][NB + 1];
    __shared__ zd X[NB][64 + 1];
    const int c0 = k + jb + blockIdx.x * 64;
    const int tid = threadIdx.x;
    for (int e = tid; e < jb * jb; e += 256) {
        int r = e / jb, c = e % jb;
        L[r][c] = A[(long)(k + r) * ld + k + c];
    }
    for (int e = tid; e < jb * 64; e += 256) {
        int r = e / 64, c = e % 64;
        X[r][c] = (c0 + c < n) ? A[(long)(k + r) * ld + c0 + c] : czero<double>();
    }
    __syncthreads();
    for (int r = 0; r < jb; ++r) {
        int cnt = (jb - r - 1) * 64;
        for (int e = tid; e < cnt; e += 256) {
            int rr = r + 1 + e / 64, c = e % 64;
            cfms(X[rr][c], L[rr][r], X[r][c]);
        }
        __syncthreads();
    }
    for (int e = tid; e < jb * 64; e += 256) {
        int r = e / 64, c = e % 64;
        if (c0 + c < n) A[(long)(k + r) * ld + c0 + c] = X[r][c];
    }
}

void lu_factor(hipStream_t st, int n, zd* M, int batch, int* ipiv, int* info, DBuf&) {
    FH_HIP(hipMemsetAsync(info, 0, sizeof(int) * batch, st));
    for (int k = 0; k < n; k += NB) {
        const int jb = std::min(NB, n - k);
        k_lu_panel<256><<<batch, 256, 0, st>>>(n, M, k, jb, ipiv, info);
        FH_LAUNCH_CHECK();
        const int rest = n - k - jb;
        if (rest > 0) {
            dim3 g(ceil_div(rest, 64), batch);
            k_lu_trsm_row<<<g, 256, 0, st>>>(n, M, k, jb);
            FH_LAUNCH_CHECK();
            // A22 -= L21 U12
            zd* L21 = M + (long)(k + jb) * n + k;
            zd* U12 = M + (long)k * n + k + jb;
            zd* A22 = M + (long)(k + jb) * n + k + jb;
            gemm<double>(st, 'N', 'N', rest, rest, jb, cx(-1.0, 0.0), L21, n, (long)n * n, U12, n, (long)n * n,
                         cx(1.0, 0.0), A22, n, (long)n * n, batch);
        }
    }
}

// ---------------------------------------------------------------------------
// solves
// ---------------------------------------------------------------------------
// row interchanges on X (n x m, ld m): forward order (k = 0..n-1) or reverse
__global__ void k_laswp(int n, const int* __restrict__ ipiv, int m, zd* __restrict__ Xall, int reverse) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    zd* X = Xall + (long)blockIdx.y * n * m;
    const int* piv = ipiv + (long)blockIdx.y * n;
    if (!reverse) {
        for (int k = 0; k < n; ++k) {
            int p = piv[k];
            if (p != k) { zd t = X[(long)k * m + c]; X[(long)k * m + c] = X[(long)p * m + c]; X[(long)p * m + c] = t; }
        }
    } else {
        for (int k = n - 1; k >= 0; --k) {
            int p = piv[k];
            if (p != k) { zd t = X[(long)k * m + c]; X[(long)k * m + c] = X[(long)p * m + c]; X[(long)p * m + c] = t; }
        }
    }
}

// Diagonal block [k, k+jb): X_k <- T_kk^{-1} X_k where T = L (unit lower),
// U (upper), U^H (lower) or L^H (unit upper) of the packed LU in M.
template <bool UPPER, bool UNIT, bool CT>
__global__ __launch_bounds__(256) void k_trsm_diag(int n, const zd* __restrict__ Mall, int k, int jb, int m,
                                                   zd* __restrict__ Xall) {
    const zd* A = Mall + (long)blockIdx.y * n * n;
    zd* X = Xall + (long)blockIdx.y * n * m;
    __shared__ zd T[NB][NB + 1];
    __shared__ zd S[NB][64 + 1];
    const int c0 = blockIdx.x * 64, tid = threadIdx.x;
    for (int e = tid; e < jb * jb; e += 256) {
        int r = e / jb, c = e % jb;
        T[r][c] = CT ? conj(A[(long)(k + c) * n + k + r]) : A[(long)(k + r) * n + k + c];
    }
    for (int e = tid; e < jb * 64; e += 256) {
        int r = e / 64, c = e % 64;
        S[r][c] = (c0 + c < m) ? X[(long)(k + r) * m + c0 + c] : czero<double>();
    }
    __syncthreads();
    if (!UPPER) {
        for (int r = 0; r < jb; ++r) {
            if (!UNIT) {
                if (tid < 64) S[r][tid] = cdiv(S[r][tid], T[r][r]);
                __syncthreads();
            }
            int cnt = (jb - r - 1) * 64;
            for (int e = tid; e < cnt; e += 256) {
                int rr = r + 1 + e / 64, c = e % 64;
                cfms(S[rr][c], T[rr][r], S[r][c]);
            }
            __syncthreads();
        }
    } else {
        for (int r = jb - 1; r >= 0; --r) {
            if (!UNIT) {
                if (tid < 64) S[r][tid] = cdiv(S[r][tid], T[r][r]);
                __syncthreads();
            }
            int cnt = r * 64;
            for (int e = tid; e < cnt; e += 256) {
                int rr = e / 64, c = e % 64;
                cfms(S[rr][c], T[rr][r], S[r][c]);
            }
            __syncthreads();
        }
    }
    for (int e = tid; e < jb * 64; e += 256) {
        int r = e / 64, c = e % 64;
        if (c0 + c < m) X[(long)(k + r) * m + c0 + c] = S[r][c];
    }
}

template <bool UPPER, bool UNIT, bool CT>
static void trsm_blocked(hipStream_t st, int n, const zd* M, int m, zd* X, int batch) {
    dim3 g(ceil_div(m, 64), batch);
    const long sM = (long)n * n, sX = (long)n * m;
    const int nblk = ceil_div(n, NB);
    for (int bi = 0; bi < nblk; ++bi) {
        const int blk = UPPER ? (nblk - 1 - bi) : bi;
        const int k = blk * NB, jb = std::min(NB, n - k);
        k_trsm_diag<UPPER, UNIT, CT><<<g, 256, 0, st>>>(n, M, k, jb, m, X);
        FH_LAUNCH_CHECK();
        if (!UPPER) {
            const int rest = n - k - jb;
            if (rest <= 0) continue;
            // X[k+jb:] -= T[k+jb:, k:k+jb] X[k:k+jb]
            if (!CT)
                gemm<double>(st, 'N', 'N', rest, m, jb, cx(-1.0, 0.0), M + (long)(k + jb) * n + k, n, sM,
                             X + (long)k * m, m, sX, cx(1.0, 0.0), X + (long)(k + jb) * m, m, sX, batch);
            else  // T = U^H: T[i][j] = conj(U[j][i]), block = (U[k:k+jb, k+jb:])^H
                gemm<double>(st, 'C', 'N', rest, m, jb, cx(-1.0, 0.0), M + (long)k * n + k + jb, n, sM,
                             X + (long)k * m, m, sX, cx(1.0, 0.0), X + (long)(k + jb) * m, m, sX, batch);
        } else {
            if (k <= 0) continue;
            // X[0:k] -= T[0:k, k:k+jb] X[k:k+jb]
            if (!CT)
                gemm<double>(st, 'N', 'N', k, m, jb, cx(-1.0, 0.0), M + k, n, sM, X + (long)k * m, m, sX,
                             cx(1.0, 0.0), X, m, sX, batch);
            else  // T = L^H: block = (L[k:k+jb, 0:k])^H
                gemm<double>(st, 'C', 'N', k, m, jb, cx(-1.0, 0.0), M + (long)k * n, n, sM, X + (long)k * m, m,
                             sX, cx(1.0, 0.0), X, m, sX, batch);
        }
    }
}

void lu_solve(hipStream_t st, char op, int n, const zd* M, const int* ipiv, int m, zd* X, int batch) {
    dim3 gs(ceil_div(m, 64), batch);
    if (op == 'N') {
        k_laswp<<<gs, 64, 0, st>>>(n, ipiv, m, X, 0);
        FH_LAUNCH_CHECK();
        trsm_blocked<false, true, false>(st, n, M, m, X, batch);   // L
        trsm_blocked<true, false, false>(st, n, M, m, X, batch);   // U
    } else {
        trsm_blocked<false, false, true>(st, n, M, m, X, batch);   // U^H
        trsm_blocked<true, true, true>(st, n, M, m, X, batch);     // L^H
        k_laswp<<<gs, 64, 0, st>>>(n, ipiv, m, X, 1);
        FH_LAUNCH_CHECK();
    }
}

}  // namespace fh
