// Grouped dense kernels (see fh_group.h): every launch works on a list of
// matrices of different sizes, so that the LU of every node of every instance
// of a batch advances one panel per launch, and the GEMM updates of all of
// them share one launch whose workgroups are spread over a flattened tile
// list.  Complex FP32 GEMMs use V_MFMA_F32_16X16X4_F32 (four real products
// per complex one); FP64 GEMMs use vector FMA (on this chip FP64 matrix and
// vector peaks are equal).
#include <cstring>
#include <type_traits>

#include "fh_group.h"
#include "fh_prof.h"

namespace fh {

typedef float v4f __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// panel factorization: columns [k, k+jb) of rows [k, n) of each listed matrix;
// pivot by |re| + |im| (lowest index on ties); interchanges on whole rows.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_gpanel(const GMat<T>* __restrict__ list) {
    const GMat<T> g = list[blockIdx.x];
    Cx<T>* A = g.M;
    const int n = g.n, k = g.k, jb = g.jb;
    const long ld = n;
    __shared__ T sv[NT];
    __shared__ int si[NT];
    const int tid = threadIdx.x;
    if (k == 0 && tid == 0) *g.info = 0;
    for (int c = k; c < k + jb; ++c) {
        T best = T(-1);
        int bi = c;
        for (int i = c + tid; i < n; i += NT) {
            const T v = cabs1(A[(long)i * ld + c]);
            if (v > best) { best = v; bi = i; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (tid < s) {
                const T o = sv[tid + s];
                const int oi = si[tid + s];
                if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
            }
            __syncthreads();
        }
        const int p = si[0];
        const T pv = sv[0];
        __syncthreads();
        if (tid == 0) {
            g.ipiv[c] = p;
            if (!(pv > T(0)) && *g.info == 0) *g.info = c + 1;
        }
        if (p != c) {
            for (int j = tid; j < n; j += NT) {
                const Cx<T> t = A[(long)c * ld + j];
                A[(long)c * ld + j] = A[(long)p * ld + j];
                A[(long)p * ld + j] = t;
            }
        }
        __syncthreads();
        if (pv > T(0)) {
            const Cx<T> dinv = cdiv(cx(T(1), T(0)), A[(long)c * ld + c]);
            for (int i = c + 1 + tid; i < n; i += NT) {
                const Cx<T> l = A[(long)i * ld + c] * dinv;
                A[(long)i * ld + c] = l;
                for (int j = c + 1; j < k + jb; ++j) cfms(A[(long)i * ld + j], l, A[(long)c * ld + j]);
            }
        }
        __syncthreads();
    }
}

// U12 = L11^{-1} A12 for rows [k, k+jb), columns [k+jb, n) in 64-wide tiles
template <typename T>
__global__ __launch_bounds__(256) void k_gtrsm_row(const GMat<T>* __restrict__ list) {
    const GMat<T> g = list[blockIdx.y];
    const int n = g.n, k = g.k, jb = g.jb;
    const int c0 = k + jb + blockIdx.x * 64;
    if (c0 >= n) return;          // uniform over the workgroup
    Cx<T>* A = g.M;
    const long ld = n;
    __shared__ Cx<T> L[GNB][GNB + 1];
    __shared__ Cx<T> X[GNB][64 + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < jb * jb; e += 256) {
        const int r = e / jb, c = e % jb;
        L[r][c] = A[(long)(k + r) * ld + k + c];
    }
    for (int e = tid; e < jb * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        X[r][c] = (c0 + c < n) ? A[(long)(k + r) * ld + c0 + c] : czero<T>();
    }
    __syncthreads();
    for (int r = 0; r < jb; ++r) {
        const int cnt = (jb - r - 1) * 64;
        for (int e = tid; e < cnt; e += 256) {
            const int rr = r + 1 + e / 64, c = e % 64;
            cfms(X[rr][c], L[rr][r], X[r][c]);
        }
        __syncthreads();
    }
    for (int e = tid; e < jb * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        if (c0 + c < n) A[(long)(k + r) * ld + c0 + c] = X[r][c];
    }
}

// row interchanges of X (n x m, ld m), forward (k ascending) or reverse
template <typename T>
__global__ void k_glaswp(const GMat<T>* __restrict__ list, int reverse) {
    const GMat<T> g = list[blockIdx.y];
    const int m = g.m;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    Cx<T>* X = g.X;
    const int n = g.n;
    for (int q = 0; q < n; ++q) {
        const int kk = reverse ? n - 1 - q : q;
        const int p = g.ipiv[kk];
        if (p != kk) {
            const Cx<T> t = X[(long)kk * m + c];
            X[(long)kk * m + c] = X[(long)p * m + c];
            X[(long)p * m + c] = t;
        }
    }
}

// diagonal block [k, k+jb) of a triangular solve on X (columns in 64-wide
// tiles): T = L (unit lower), U (upper), U^H (lower) or L^H (unit upper)
template <typename T, bool UPPER, bool UNIT, bool CT>
__global__ __launch_bounds__(256) void k_gdiag(const GMat<T>* __restrict__ list) {
    const GMat<T> g = list[blockIdx.y];
    const int n = g.n, k = g.k, jb = g.jb, m = g.m;
    if ((int)blockIdx.x * 64 >= m) return;     // uniform over the workgroup
    const Cx<T>* A = g.M;
    Cx<T>* X = g.X;
    __shared__ Cx<T> Tm[GNB][GNB + 1];
    __shared__ Cx<T> S[GNB][64 + 1];
    const int c0 = blockIdx.x * 64, tid = threadIdx.x;
    for (int e = tid; e < jb * jb; e += 256) {
        const int r = e / jb, c = e % jb;
        Tm[r][c] = CT ? conj(A[(long)(k + c) * n + k + r]) : A[(long)(k + r) * n + k + c];
    }
    for (int e = tid; e < jb * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        S[r][c] = (c0 + c < m) ? X[(long)(k + r) * m + c0 + c] : czero<T>();
    }
    __syncthreads();
    for (int q = 0; q < jb; ++q) {
        const int r = UPPER ? jb - 1 - q : q;
        if (!UNIT) {
            if (tid < 64) S[r][tid] = cdiv(S[r][tid], Tm[r][r]);
            __syncthreads();
        }
        const int cnt = (UPPER ? r : jb - r - 1) * 64;
        for (int e = tid; e < cnt; e += 256) {
            const int rr = (UPPER ? 0 : r + 1) + e / 64, c = e % 64;
            cfms(S[rr][c], Tm[rr][r], S[r][c]);
        }
        __syncthreads();
    }
    for (int e = tid; e < jb * 64; e += 256) {
        const int r = e / 64, c = e % 64;
        if (c0 + c < m) X[(long)(k + r) * m + c0 + c] = S[r][c];
    }
}

// ---------------------------------------------------------------------------
// grouped GEMM: blockIdx.x -> (item, tile) by binary search of tile0
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int find_item(const GItem<T>* __restrict__ items, int nitems, int t) {
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// vector-FMA version (any T): (16 RA) x (16 RB) tile, RA x RB complex
// micro-tile per thread (64 x 64 in general; 128 x 32 when every item of the
// launch has at most 32 columns, so that no FMA works on padding)
template <typename T, bool CA, int RA, int RB>
__global__ __launch_bounds__(256) void k_ggemm_fma(const GItem<T>* __restrict__ items, int nitems) {
    constexpr int TM = 16 * RA, TN = 16 * RB;
    const int t = blockIdx.x;
    const GItem<T> it = items[find_item(items, nitems, t)];
    const int tl = t - it.tile0;
    const int m0 = (tl / it.tiles_n) * TM, n0 = (tl % it.tiles_n) * TN;
    constexpr int KT = 16;
    __shared__ Cx<T> As[KT][TM + 1];
    __shared__ Cx<T> Bs[KT][TN + 1];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    Cx<T> acc[RA][RB];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) acc[a][b] = czero<T>();
    // the next K tile is loaded into registers while the FMAs work on the
    // current one from LDS
    Cx<T> ra[RA], rb[RB];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < RA; ++q) {
            const int e = tid + 256 * q;
            int i, kk;
            if (!CA) { i = e / KT; kk = e % KT; } else { kk = e / TM; i = e % TM; }
            const int gi = m0 + i, gk = k0 + kk;
            Cx<T> v = czero<T>();
            if (gi < it.M && gk < it.K) v = CA ? conj(it.A[(long)gk * it.lda + gi]) : it.A[(long)gi * it.lda + gk];
            ra[q] = v;
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int e = tid + 256 * q;
            const int kb = e / TN, j = e % TN;
            Cx<T> u = czero<T>();
            if (n0 + j < it.N && k0 + kb < it.K) u = it.B[(long)(k0 + kb) * it.ldb + n0 + j];
            rb[q] = u;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int q = 0; q < RA; ++q) {
            const int e = tid + 256 * q;
            int i, kk;
            if (!CA) { i = e / KT; kk = e % KT; } else { kk = e / TM; i = e % TM; }
            As[kk][i] = ra[q];
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int e = tid + 256 * q;
            Bs[e / TN][e % TN] = rb[q];
        }
    };
    load(0);
    store();
    __syncthreads();
    for (int k0 = 0; k0 < it.K; k0 += KT) {
        const bool more = k0 + KT < it.K;
        if (more) load(k0 + KT);
#pragma unroll 2
        for (int kk = 0; kk < KT; ++kk) {
            Cx<T> av[RA], bv[RB];
#pragma unroll
            for (int a = 0; a < RA; ++a) av[a] = As[kk][ty + 16 * a];
#pragma unroll
            for (int b = 0; b < RB; ++b) bv[b] = Bs[kk][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < RA; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b) cfma(acc[a][b], av[a], bv[b]);
        }
        __syncthreads();
        if (more) {
            store();
            __syncthreads();
        }
    }
#pragma unroll
    for (int a = 0; a < RA; ++a) {
        const int gi = m0 + ty + 16 * a;
        if (gi >= it.M) continue;
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int gj = n0 + tx + 16 * b;
            if (gj >= it.N) continue;
            Cx<T>& c = it.C[(long)gi * it.ldc + gj];
            Cx<T> r = it.beta1 ? c : czero<T>();
            cfma(r, it.alpha, acc[a][b]);
            c = r;
        }
    }
}

// complex FP32 on MFMA.  TS = 64: the 4 waves cover 2 x 2 quadrants of 32 x 32,
// each as 2 x 2 blocks of 16 x 16; TS = 32: each wave one 16 x 16 block.
// Lane l of a 16x16x4 MFMA supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// its 4 results are D[4 (l / 16) + v][l % 16].
template <bool CA, int TS>
__global__ __launch_bounds__(256) void k_ggemm_mfma(const GItem<float>* __restrict__ items, int nitems) {
    const int t = blockIdx.x;
    const GItem<float> it = items[find_item(items, nitems, t)];
    const int tl = t - it.tile0;
    const int m0 = (tl / it.tiles_n) * TS, n0 = (tl % it.tiles_n) * TS;
    constexpr int KT = 16;
    constexpr int NBK = TS / 32;          // 16x16 blocks per wave along each dimension
    constexpr int NE = TS * KT / 256;     // tile entries of A (and of B) per thread
    // two stages: the next K tile is loaded into registers while the MFMAs
    // work on the current one, then stored into the other stage (one
    // barrier per K tile)
    __shared__ float Ar[2][TS][KT + 1], Ai[2][TS][KT + 1];
    __shared__ float Br[2][KT][TS + 1], Bi[2][KT][TS + 1];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * (TS / 2), wc = (wave & 1) * (TS / 2);
    const int li = lane & 15, lk = lane >> 4;
    v4f accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            accr[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
            acci[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    cf ra[NE], rb[NE];
    auto load = [&](int k0) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = tid + 256 * q;
            int i, kk;
            if (!CA) { i = e / KT; kk = e % KT; } else { kk = e / TS; i = e % TS; }
            const int gi = m0 + i, gk = k0 + kk;
            cf v = czero<float>();
            if (gi < it.M && gk < it.K) v = CA ? conj(it.A[(long)gk * it.lda + gi]) : it.A[(long)gi * it.lda + gk];
            ra[q] = v;
            const int kb = e / TS, j = e % TS;
            cf u = czero<float>();
            if (n0 + j < it.N && k0 + kb < it.K) u = it.B[(long)(k0 + kb) * it.ldb + n0 + j];
            rb[q] = u;
        }
    };
    auto store = [&](int st) {
#pragma unroll
        for (int q = 0; q < NE; ++q) {
            const int e = tid + 256 * q;
            int i, kk;
            if (!CA) { i = e / KT; kk = e % KT; } else { kk = e / TS; i = e % TS; }
            Ar[st][i][kk] = ra[q].re;
            Ai[st][i][kk] = ra[q].im;
            const int kb = e / TS, j = e % TS;
            Br[st][kb][j] = rb[q].re;
            Bi[st][kb][j] = rb[q].im;
        }
    };
    load(0);
    store(0);
    __syncthreads();
    int st = 0;
    for (int k0 = 0; k0 < it.K; k0 += KT) {
        const bool more = k0 + KT < it.K;
        if (more) load(k0 + KT);
#pragma unroll
        for (int kq = 0; kq < KT; kq += 4) {
            float are[2], aim[2], bre[2], bim[2];
#pragma unroll
            for (int a = 0; a < NBK; ++a) {
                are[a] = Ar[st][wr + 16 * a + li][kq + lk];
                aim[a] = Ai[st][wr + 16 * a + li][kq + lk];
            }
#pragma unroll
            for (int b = 0; b < NBK; ++b) {
                bre[b] = Br[st][kq + lk][wc + 16 * b + li];
                bim[b] = Bi[st][kq + lk][wc + 16 * b + li];
            }
#pragma unroll
            for (int a = 0; a < NBK; ++a)
#pragma unroll
                for (int b = 0; b < NBK; ++b) {
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[a], bre[b], accr[a][b], 0, 0, 0);
                    accr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-aim[a], bim[b], accr[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(are[a], bim[b], acci[a][b], 0, 0, 0);
                    acci[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aim[a], bre[b], acci[a][b], 0, 0, 0);
                }
        }
        if (more) store(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
#pragma unroll
    for (int a = 0; a < NBK; ++a)
#pragma unroll
        for (int b = 0; b < NBK; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gi = m0 + wr + 16 * a + 4 * lk + v;
                const int gj = n0 + wc + 16 * b + li;
                if (gi < it.M && gj < it.N) {
                    cf& c = it.C[(long)gi * it.ldc + gj];
                    cf r = it.beta1 ? c : czero<float>();
                    cfma(r, it.alpha, cf{accr[a][b][v], acci[a][b][v]});
                    c = r;
                }
            }
}

// ---------------------------------------------------------------------------
// elementwise work over a set of blocks (block s: len[s] entries at off[s])
// ---------------------------------------------------------------------------
// R_s = B_s - z_s X_s   (z_s as given; X == nullptr: R_s = B_s)
__global__ void k_set_resid_init(const long* __restrict__ off, const int* __restrict__ len, const zd* __restrict__ z,
                                 const zd* __restrict__ Bv, const zd* __restrict__ X, zd* __restrict__ R) {
    const int s = blockIdx.y;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len[s]) return;
    const long q = off[s] + e;
    zd r = Bv[q];
    if (X) cfms(r, z[s], X[q]);
    R[q] = r;
}

// out[s * mmax + c] = || column c of block s ||_2  (block s: n[s] x m[s], ld m[s]);
// one workgroup per block: column c is summed by the threads t with
// t % w == c over row strides of 256 / w (w = columns per pass), then reduced in LDS
__global__ __launch_bounds__(256) void k_set_colnorm(const long* __restrict__ off, const int* __restrict__ n,
                                                     const int* __restrict__ m, int mmax, const zd* __restrict__ V,
                                                     double* __restrict__ out) {
    __shared__ double red[256];
    const int s = blockIdx.x, tid = threadIdx.x;
    const int ms = m[s], ns = n[s];
    const zd* v = V + off[s];
    for (int c0 = 0; c0 < mmax; c0 += 64) {
        const int w = 64;                       // columns per pass
        const int c = c0 + (tid % w), g = tid / w, ng = 256 / w;
        double a = 0.0;
        if (c < ms)
            for (int i = g; i < ns; i += ng) a += abs2(v[(long)i * ms + c]);
        red[tid] = a;
        __syncthreads();
        if (g == 0 && c < mmax) {
            double t = 0.0;
            for (int q = 0; q < ng; ++q) t += red[q * w + (tid % w)];
            out[(long)s * mmax + c] = sqrt(t);
        }
        __syncthreads();
    }
}

__global__ void k_add_cast(long len, const cf* __restrict__ x, zd* __restrict__ y) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) y[e] = y[e] + zd{(double)x[e].re, (double)x[e].im};
}

void set_resid_init(hipStream_t st, int count, int maxlen, const long* off, const int* len, const zd* z, const zd* Bv,
                    const zd* X, zd* R) {
    if (count <= 0 || maxlen <= 0) return;
    k_set_resid_init<<<dim3(ceil_div(maxlen, 256), count), 256, 0, st>>>(off, len, z, Bv, X, R);
    FH_LAUNCH_CHECK();
}
void set_colnorm(hipStream_t st, int count, int mmax, const long* off, const int* n, const int* m, const zd* V,
                 double* out) {
    if (count <= 0) return;
    k_set_colnorm<<<count, 256, 0, st>>>(off, n, m, mmax, V, out);
    FH_LAUNCH_CHECK();
}
// X_s = I (n_s x n_s at element offset off[s]); X must be zero on entry
__global__ void k_set_identity(const long* __restrict__ off, const int* __restrict__ n, cf* __restrict__ X) {
    const int s = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int ns = n[s];
    if (i < ns) X[off[s] + (long)i * ns + i] = cf{1.0f, 0.0f};
}
void set_identity(hipStream_t st, int count, int nmax, const long* off, const int* n, cf* X) {
    if (count <= 0 || nmax <= 0) return;
    k_set_identity<<<dim3(ceil_div(nmax, 256), count), 256, 0, st>>>(off, n, X);
    FH_LAUNCH_CHECK();
}

void add_cast(hipStream_t st, long len, const cf* x, zd* y) {
    if (len <= 0) return;
    k_add_cast<<<ceil_div(len, 256), 256, 0, st>>>(len, x, y);
    FH_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
static int tile_of(int tile) { return tile == GTILE_32 ? 32 : 64; }

template <typename T>
static void launch_gemm(hipStream_t st, const GOp& op, const void* list, int tile);

template <>
void launch_gemm<double>(hipStream_t st, const GOp& op, const void* list, int) {
    const GItem<double>* it = (const GItem<double>*)list;
    const bool c = op.kind == GOP_GEMM_C;
    if (op.narrow) {
        if (c) k_ggemm_fma<double, true, 8, 2><<<op.tiles, 256, 0, st>>>(it, op.count);
        else k_ggemm_fma<double, false, 8, 2><<<op.tiles, 256, 0, st>>>(it, op.count);
    } else {
        if (c) k_ggemm_fma<double, true, 4, 4><<<op.tiles, 256, 0, st>>>(it, op.count);
        else k_ggemm_fma<double, false, 4, 4><<<op.tiles, 256, 0, st>>>(it, op.count);
    }
    FH_LAUNCH_CHECK();
}

template <>
void launch_gemm<float>(hipStream_t st, const GOp& op, const void* list, int tile) {
    const GItem<float>* it = (const GItem<float>*)list;
    const bool c = op.kind == GOP_GEMM_C;
    if (tile == GTILE_32) {
        if (c) k_ggemm_mfma<true, 32><<<op.tiles, 256, 0, st>>>(it, op.count);
        else k_ggemm_mfma<false, 32><<<op.tiles, 256, 0, st>>>(it, op.count);
    } else {
        if (c) k_ggemm_mfma<true, 64><<<op.tiles, 256, 0, st>>>(it, op.count);
        else k_ggemm_mfma<false, 64><<<op.tiles, 256, 0, st>>>(it, op.count);
    }
    FH_LAUNCH_CHECK();
}

template <typename T>
void GroupPlan<T>::run(hipStream_t st) const {
    const char* base = (const char*)buf.p;
    for (const GOp& op : ops) {
        const void* list = base + op.off;
        const GMat<T>* ml = (const GMat<T>*)list;
        switch (op.kind) {
            case GOP_PANEL:
                k_gpanel<T, 256><<<op.count, 256, 0, st>>>(ml);
                break;
            case GOP_TRSM_ROW:
                k_gtrsm_row<T><<<dim3(op.tiles, op.count), 256, 0, st>>>(ml);
                break;
            case GOP_GEMM_N:
            case GOP_GEMM_C: {
                hipEvent_t ev = prof_begin(st);
                launch_gemm<T>(st, op, list, tile);
                if (ev)
                    prof_end(st, ev, std::is_same<T, float>::value ? (tile == GTILE_32 ? "ggemm_c64_mfma32" : "ggemm_c64_mfma64")
                                                                   : "ggemm_c128_fma",
                             op.bytes, op.flops);
                break;
            }
            case GOP_LASWP_F:
            case GOP_LASWP_R:
                k_glaswp<T><<<dim3(ceil_div(op.mcols, 64), op.count), 64, 0, st>>>(ml, op.kind == GOP_LASWP_R);
                break;
            case GOP_DIAG: {
                const dim3 g(ceil_div(op.mcols, 64), op.count);
                if (op.diag_variant == 0) k_gdiag<T, false, true, false><<<g, 256, 0, st>>>(ml);
                else if (op.diag_variant == 1) k_gdiag<T, true, false, false><<<g, 256, 0, st>>>(ml);
                else if (op.diag_variant == 2) k_gdiag<T, false, false, true><<<g, 256, 0, st>>>(ml);
                else k_gdiag<T, true, true, true><<<g, 256, 0, st>>>(ml);
                break;
            }
        }
        FH_LAUNCH_CHECK();
    }
}

// host-side builder: work lists appended to one byte vector, uploaded once
namespace {
struct Builder {
    std::vector<char> bytes;
    template <typename E>
    size_t add(const std::vector<E>& v) {
        size_t off = (bytes.size() + 255) / 256 * 256;
        bytes.resize(off + sizeof(E) * v.size());
        std::memcpy(bytes.data() + off, v.data(), sizeof(E) * v.size());
        return off;
    }
};

template <typename T>
void finish(GroupPlan<T>& plan, Builder& b) {
    void* d = plan.buf.ensure(std::max<size_t>(256, b.bytes.size()));
    if (!b.bytes.empty()) FH_HIP(hipMemcpy(d, b.bytes.data(), b.bytes.size(), hipMemcpyHostToDevice));
}

template <typename T>
void add_gemm(GroupPlan<T>& plan, Builder& bld, bool conjA, std::vector<GItem<T>>& items, int tile) {
    // FP64 (vector FMA): 128 x 32 tiles when no item has more than 32 columns
    bool narrow = !std::is_same<T, float>::value;
    for (const GItem<T>& it : items)
        if (it.M > 0 && it.N > 32) narrow = false;
    const int tm = (std::is_same<T, float>::value) ? tile_of(tile) : (narrow ? 128 : 64);
    const int tn = (std::is_same<T, float>::value) ? tile_of(tile) : (narrow ? 32 : 64);
    std::vector<GItem<T>> keep;
    int tiles = 0;
    for (GItem<T> it : items) {
        if (it.M <= 0 || it.N <= 0) continue;
        it.tiles_n = (int)ceil_div(it.N, tn);
        it.tile0 = tiles;
        tiles += (int)ceil_div(it.M, tm) * it.tiles_n;
        keep.push_back(it);
    }
    if (keep.empty()) return;
    GOp op{};
    op.narrow = narrow ? 1 : 0;
    for (const auto& it : keep) {
        op.flops += 8.0 * it.M * it.N * it.K;
        op.bytes += (double)sizeof(Cx<T>) * ((double)it.M * it.K + (double)it.K * it.N + 2.0 * it.M * it.N);
    }
    op.kind = conjA ? GOP_GEMM_C : GOP_GEMM_N;
    op.off = bld.add(keep);
    op.count = (int)keep.size();
    op.tiles = tiles;
    plan.ops.push_back(op);
}
}  // namespace

template <typename T>
void group_gemm_plan(GroupPlan<T>& plan, bool conjA, std::vector<GItem<T>> items, int tile) {
    plan.ops.clear();
    plan.tile = tile;
    Builder b;
    add_gemm(plan, b, conjA, items, tile);
    finish(plan, b);
}

template <typename T>
void group_lu_plan(GroupPlan<T>& plan, int count, Cx<T>* const* M, const int* n, int* const* ipiv,
                   int* const* info, int tile) {
    plan.ops.clear();
    plan.tile = tile;
    Builder b;
    int nmax = 0;
    for (int i = 0; i < count; ++i) nmax = std::max(nmax, n[i]);
    for (int k = 0; k < nmax; k += GNB) {
        std::vector<GMat<T>> act;
        std::vector<GItem<T>> items;
        int maxrest = 0;
        for (int i = 0; i < count; ++i) {
            if (n[i] <= k) continue;
            const int jb = std::min(GNB, n[i] - k), rest = n[i] - k - jb;
            act.push_back(GMat<T>{M[i], ipiv[i], info[i], nullptr, n[i], k, jb, 0});
            maxrest = std::max(maxrest, rest);
            if (rest > 0) {
                Cx<T>* A = M[i];
                const long ld = n[i];
                items.push_back(GItem<T>{A + (k + jb) * ld + k, A + k * ld + k + jb, A + (k + jb) * ld + k + jb, rest,
                                         rest, jb, n[i], n[i], n[i], 0, 0, cx(T(-1), T(0)), 1});
            }
        }
        GOp p{};
        p.kind = GOP_PANEL;
        p.off = b.add(act);
        p.count = (int)act.size();
        plan.ops.push_back(p);
        if (maxrest > 0) {
            std::vector<GMat<T>> tr;
            for (const auto& g : act)
                if (g.n - g.k - g.jb > 0) tr.push_back(g);
            GOp r{};
            r.kind = GOP_TRSM_ROW;
            r.off = b.add(tr);
            r.count = (int)tr.size();
            r.tiles = (int)ceil_div(maxrest, 64);
            plan.ops.push_back(r);
            add_gemm(plan, b, false, items, tile);
        }
    }
    finish(plan, b);
}

template <typename T>
void group_solve_plan(GroupPlan<T>& plan, char opc, int count, Cx<T>* const* M, const int* n, int* const* ipiv,
                      Cx<T>* const* X, const int* mm, int tile) {
    plan.ops.clear();
    plan.tile = tile;
    Builder b;
    int nmax = 0, mmax = 0;
    for (int i = 0; i < count; ++i) {
        nmax = std::max(nmax, n[i]);
        mmax = std::max(mmax, mm[i]);
    }
    const int nblk = (int)ceil_div(nmax, GNB);
    std::vector<GMat<T>> all;
    for (int i = 0; i < count; ++i)
        if (mm[i] > 0) all.push_back(GMat<T>{M[i], ipiv[i], nullptr, X[i], n[i], 0, 0, mm[i]});
    if (all.empty()) {
        finish(plan, b);
        return;
    }
    auto laswp = [&](bool rev) {
        GOp o{};
        o.kind = rev ? GOP_LASWP_R : GOP_LASWP_F;
        o.off = b.add(all);
        o.count = (int)all.size();
        o.mcols = mmax;
        plan.ops.push_back(o);
    };
    // one sweep: variant 0 L, 1 U, 2 U^H, 3 L^H; lower sweeps go by ascending blocks
    auto sweep = [&](int variant) {
        const bool upper = (variant == 1 || variant == 3);
        const bool ct = (variant >= 2);
        for (int q = 0; q < nblk; ++q) {
            std::vector<GMat<T>> d;
            std::vector<GItem<T>> items;
            for (int i = 0; i < count; ++i) {
                if (mm[i] <= 0) continue;
                const int m = mm[i];
                const int nb_i = (int)ceil_div(n[i], GNB);
                // lower sweeps: block q; upper sweeps: block nb_i-1-(q - (nblk - nb_i)) so that
                // every matrix runs its blocks from its own last one down
                int blk;
                if (!upper) {
                    if (q >= nb_i) continue;
                    blk = q;
                } else {
                    const int qq = q - (nblk - nb_i);
                    if (qq < 0) continue;
                    blk = nb_i - 1 - qq;
                }
                const int k = blk * GNB, jb = std::min(GNB, n[i] - k);
                d.push_back(GMat<T>{M[i], ipiv[i], nullptr, X[i], n[i], k, jb, m});
                Cx<T>* A = M[i];
                const long ld = n[i];
                if (!upper) {
                    const int rest = n[i] - k - jb;
                    if (rest <= 0) continue;
                    // X[k+jb:] -= T[k+jb:, k:k+jb] X[k:k+jb]
                    const Cx<T>* Ab = ct ? A + k * ld + k + jb : A + (k + jb) * ld + k;
                    items.push_back(GItem<T>{Ab, X[i] + (long)k * m, X[i] + (long)(k + jb) * m, rest, m, jb, n[i], m,
                                             m, 0, 0, cx(T(-1), T(0)), 1});
                } else {
                    if (k <= 0) continue;
                    // X[0:k] -= T[0:k, k:k+jb] X[k:k+jb]
                    const Cx<T>* Ab = ct ? A + k * ld : A + k;
                    items.push_back(GItem<T>{Ab, X[i] + (long)k * m, X[i], k, m, jb, n[i], m, m, 0, 0,
                                             cx(T(-1), T(0)), 1});
                }
            }
            if (d.empty()) continue;
            GOp o{};
            o.kind = GOP_DIAG;
            o.diag_variant = variant;
            o.off = b.add(d);
            o.count = (int)d.size();
            o.mcols = mmax;
            plan.ops.push_back(o);
            add_gemm(plan, b, ct, items, tile);
        }
    };
    if (opc == 'N') {
        laswp(false);
        sweep(0);
        sweep(1);
    } else {
        sweep(2);
        sweep(3);
        laswp(true);
    }
    finish(plan, b);
}

template struct GroupPlan<double>;
template struct GroupPlan<float>;
template void group_lu_plan<double>(GroupPlan<double>&, int, zd* const*, const int*, int* const*, int* const*, int);
template void group_lu_plan<float>(GroupPlan<float>&, int, cf* const*, const int*, int* const*, int* const*, int);
template void group_solve_plan<double>(GroupPlan<double>&, char, int, zd* const*, const int*, int* const*,
                                       zd* const*, const int*, int);
template void group_solve_plan<float>(GroupPlan<float>&, char, int, cf* const*, const int*, int* const*,
                                      cf* const*, const int*, int);
template void group_gemm_plan<double>(GroupPlan<double>&, bool, std::vector<GItem<double>>, int);
template void group_gemm_plan<float>(GroupPlan<float>&, bool, std::vector<GItem<float>>, int);

}  // namespace fh
