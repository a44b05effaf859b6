// Sparse kernels of the iterative contour filter: CSR operator products with
// a fused shift, ILU(0) factorization and level-scheduled triangular sweeps
// (both the (LU)^{-1} and the (LU)^{-H} application of one factorization),
// and the column-batched GMRES building blocks (classical Gram-Schmidt with
// re-orthogonalization, Givens updates, solution update).
//
// Block vectors of a batch are stored system-major: system s occupies the
// n x m row-major block at offset s*n*m, so the m right-hand sides of one
// system are contiguous within a row and every row access is coalesced.
#include "fh_sparse.h"
#include <string>

namespace fh {

// ---------------------------------------------------------------------------
// small helpers for real/complex operator values
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void mac_val(Cx<T>& acc, T v, Cx<T> x, bool) {
    acc.re = fma(v, x.re, acc.re);
    acc.im = fma(v, x.im, acc.im);
}
template <typename T>
__device__ __forceinline__ void mac_val(Cx<T>& acc, Cx<T> v, Cx<T> x, bool conjv) {
    if (conjv) cfma_conj(acc, v, x); else cfma(acc, v, x);
}

// ---------------------------------------------------------------------------
// Out_s = alpha * (sh_s X_s - op(A) X_s) + Yadd_s      (op(A): A or A^H via the
// transposed CSR, conj applied for complex values when CONJ)
// block (m, ry), grid (ceil(n/ry), nsys)
// ---------------------------------------------------------------------------
template <typename T, typename TA, bool CONJ>
__global__ void k_spmm(int n, int m, const int* __restrict__ rowptr, const int* __restrict__ col,
                       const TA* __restrict__ val, const Cx<T>* __restrict__ shifts, T alpha,
                       const Cx<T>* __restrict__ X, const Cx<T>* __restrict__ Yadd, Cx<T>* __restrict__ Out) {
    const int r = blockIdx.x * blockDim.y + threadIdx.y;
    const int c = threadIdx.x;
    if (r >= n) return;
    const int s = blockIdx.y;
    const long base = (long)s * n * m;
    const Cx<T>* Xs = X + base;
    Cx<T> acc = czero<T>();
    const int p1 = rowptr[r + 1];
    for (int p = rowptr[r]; p < p1; ++p) mac_val(acc, val[p], Xs[(long)col[p] * m + c], CONJ);
    Cx<T> res = shifts ? shifts[s] * Xs[(long)r * m + c] : czero<T>();
    res = alpha * (res - acc);
    if (Yadd) res = res + Yadd[base + (long)r * m + c];
    Out[base + (long)r * m + c] = res;
}

// Same product for rows of at most SL entries (column blocks of >= 16 columns):
// the block first stages its rows' entries in LDS as a padded SL-slot table
// (empty slots point at the row itself with weight zero), then every thread
// issues the gathers of its RPT rows together, so that a wave keeps RPT x SL
// independent loads in flight instead of walking one row's chain of
// dependent loads (row pointer, column index, then the gathered value).
// A workgroup covers cb of the m columns of a system (blockIdx.y = system *
// ncb + column block; the last block may be partial) and ry * RPT rows:
// block (cb, ry), grid (ceil(n / (ry RPT)), nsys * ncb); rows r0 + ty + j ry.
template <typename T, typename TA, bool CONJ, int SL, int RPT>
__global__ __launch_bounds__(256) void k_spmm_rows(int n, int m, int cb, int ncb, const int* __restrict__ rowptr,
                                                   const int* __restrict__ col, const TA* __restrict__ val,
                                                   const Cx<T>* __restrict__ shifts, T alpha,
                                                   const Cx<T>* __restrict__ X, const Cx<T>* __restrict__ Yadd,
                                                   Cx<T>* __restrict__ Out) {
    constexpr int MAXR = 16 * RPT;                    // ry <= 16 (cb >= 16)
    __shared__ int s_col[MAXR * SL];
    __shared__ TA s_val[MAXR * SL];
    const int tx = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const int rows = ry * RPT;
    // Workgroups are dealt round-robin to the 8 XCDs (one L2 each): give each
    // XCD a contiguous range of row blocks, so that the gathered neighbour rows
    // (up to a grid line away) are read from the L2 that fetched them last
    long lin = blockIdx.x + (long)blockIdx.y * gridDim.x;
    const long G = (long)gridDim.x * gridDim.y;
    if (G % 8 == 0) lin = (lin % 8) * (G / 8) + lin / 8;
    const int bx = (int)(lin % gridDim.x), by = (int)(lin / gridDim.x);
    const int r0 = bx * rows;
    const int s = by / ncb;
    const int c = (by % ncb) * cb + tx;
    const bool act = c < m;
    const int tid = ty * cb + tx, nt = cb * ry;
    for (int idx = tid; idx < rows * SL; idx += nt) {
        const int rl = idx / SL, q = idx - rl * SL;
        const int r = r0 + rl;
        int cc = 0;
        TA vv{};
        if (r < n) {
            const int p = rowptr[r] + q;
            cc = r;
            if (p < rowptr[r + 1]) { cc = col[p]; vv = val[p]; }
        }
        s_col[idx] = cc;
        s_val[idx] = vv;
    }
    __syncthreads();
    if (!act) return;
    const long base = (long)s * n * m;
    const Cx<T>* Xs = X + base;
    Cx<T> xv[RPT][SL];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rl = ty + j * ry;
#pragma unroll
        for (int q = 0; q < SL; ++q) xv[j][q] = Xs[(long)s_col[rl * SL + q] * m + c];
    }
    const Cx<T> sh = shifts ? shifts[s] : czero<T>();
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rl = ty + j * ry;
        const int r = r0 + rl;
        Cx<T> acc = czero<T>();
#pragma unroll
        for (int q = 0; q < SL; ++q) mac_val(acc, s_val[rl * SL + q], xv[j][q], CONJ);
        if (r < n) {
            Cx<T> res = shifts ? sh * Xs[(long)r * m + c] : czero<T>();
            res = alpha * (res - acc);
            if (Yadd) res = res + Yadd[base + (long)r * m + c];
            Out[base + (long)r * m + c] = res;
        }
    }
}

// Complex FP32 with an even column count: the same kernel with two adjacent
// columns per lane (16-byte loads and stores, half the memory instructions).
// cb2 column pairs per workgroup, blockDim (cb2, 256 / cb2).
__device__ __forceinline__ float4 pair_of(Cx<float> a, Cx<float> b) { return make_float4(a.re, a.im, b.re, b.im); }
template <typename TA, bool CONJ, int SL, int RPT>
__global__ __launch_bounds__(256) void k_spmm_rows2(int n, int m2, int cb2, int ncb, const int* __restrict__ rowptr,
                                                    const int* __restrict__ col, const TA* __restrict__ val,
                                                    const Cx<float>* __restrict__ shifts, float alpha,
                                                    const float4* __restrict__ X, const float4* __restrict__ Yadd,
                                                    float4* __restrict__ Out) {
    constexpr int MAXR = 32 * RPT;                    // ry <= 32 (cb2 >= 8)
    __shared__ int s_col[MAXR * SL];
    __shared__ TA s_val[MAXR * SL];
    const int tx = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const int rows = ry * RPT;
    long lin = blockIdx.x + (long)blockIdx.y * gridDim.x;   // XCD-contiguous row blocks, as k_spmm_rows
    const long G = (long)gridDim.x * gridDim.y;
    if (G % 8 == 0) lin = (lin % 8) * (G / 8) + lin / 8;
    const int bx = (int)(lin % gridDim.x), by = (int)(lin / gridDim.x);
    const int r0 = bx * rows;
    const int s = by / ncb;
    const int c = (by % ncb) * cb2 + tx;              // column pair
    const bool act = c < m2;
    const int tid = ty * cb2 + tx, nt = cb2 * ry;
    for (int idx = tid; idx < rows * SL; idx += nt) {
        const int rl = idx / SL, q = idx - rl * SL;
        const int r = r0 + rl;
        int cc = 0;
        TA vv{};
        if (r < n) {
            const int p = rowptr[r] + q;
            cc = r;
            if (p < rowptr[r + 1]) { cc = col[p]; vv = val[p]; }
        }
        s_col[idx] = cc;
        s_val[idx] = vv;
    }
    __syncthreads();
    if (!act) return;
    const long base = (long)s * n * m2;
    const float4* Xs = X + base;
    float4 xv[RPT][SL];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rl = ty + j * ry;
#pragma unroll
        for (int q = 0; q < SL; ++q) xv[j][q] = Xs[(long)s_col[rl * SL + q] * m2 + c];
    }
    const Cx<float> sh = shifts ? shifts[s] : czero<float>();
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        const int rl = ty + j * ry;
        const int r = r0 + rl;
        Cx<float> a0 = czero<float>(), a1 = czero<float>();
#pragma unroll
        for (int q = 0; q < SL; ++q) {
            const float4 x = xv[j][q];
            mac_val(a0, s_val[rl * SL + q], Cx<float>{x.x, x.y}, CONJ);
            mac_val(a1, s_val[rl * SL + q], Cx<float>{x.z, x.w}, CONJ);
        }
        if (r < n) {
            Cx<float> r0v = czero<float>(), r1v = czero<float>();
            if (shifts) {
                const float4 xr = Xs[(long)r * m2 + c];
                r0v = sh * Cx<float>{xr.x, xr.y};
                r1v = sh * Cx<float>{xr.z, xr.w};
            }
            r0v = alpha * (r0v - a0);
            r1v = alpha * (r1v - a1);
            float4 o = pair_of(r0v, r1v);
            if (Yadd) {
                const float4 y = Yadd[base + (long)r * m2 + c];
                o = make_float4(o.x + y.x, o.y + y.y, o.z + y.z, o.w + y.w);
            }
            Out[base + (long)r * m2 + c] = o;
        }
    }
}

// column block of k_spmm_rows: all m columns when they divide 256 (one or
// more rows per wave), else the largest of 64, 32, 16 that divides m, else 32
// with a partial last block
static int spmm_colblock(int m) {
    if (m <= 256 && 256 % m == 0) return m;
    for (int cb : {64, 32, 16})
        if (m % cb == 0) return cb;
    return 32;
}

template <typename T, typename TA, bool CONJ, int SL, int RPT>
static void spmm_rows_launch(hipStream_t st, int n, int m, int nsys, const CsrDev& A, const TA* v,
                             const Cx<T>* shifts, T alpha, const Cx<T>* X, const Cx<T>* Yadd, Cx<T>* Out) {
    const int cb = spmm_colblock(m), ncb = ceil_div(m, cb);
    const int ry = 256 / cb;
    dim3 blk(cb, ry), grid(ceil_div(n, ry * RPT), nsys * ncb);
    k_spmm_rows<T, TA, CONJ, SL, RPT><<<grid, blk, 0, st>>>(n, m, cb, ncb, A.rowptr, A.col, v, shifts, alpha, X, Yadd,
                                                            Out);
}

template <typename TA, bool CONJ, int SL, int RPT>
static void spmm_rows2_launch(hipStream_t st, int n, int m, int nsys, const CsrDev& A, const TA* v,
                              const Cx<float>* shifts, float alpha, const Cx<float>* X, const Cx<float>* Yadd,
                              Cx<float>* Out) {
    const int m2 = m / 2, cb2 = spmm_colblock(m2), ncb = ceil_div(m2, cb2);
    const int ry = 256 / cb2;
    dim3 blk(cb2, ry), grid(ceil_div(n, ry * RPT), nsys * ncb);
    k_spmm_rows2<TA, CONJ, SL, RPT><<<grid, blk, 0, st>>>(n, m2, cb2, ncb, A.rowptr, A.col, v, shifts, alpha,
                                                          (const float4*)X, (const float4*)Yadd, (float4*)Out);
}

template <typename T, typename TA, bool CONJ>
static bool spmm_rows(hipStream_t st, int n, int m, int nsys, const CsrDev& A, const TA* v, const Cx<T>* shifts,
                      T alpha, const Cx<T>* X, const Cx<T>* Yadd, Cx<T>* Out) {
    // complex FP32, even m with column-pair blocks of at least 8 pairs, rows of
    // at most 5 entries: two columns per lane
    if constexpr (sizeof(T) == 4) {
        static int on = -1;
        if (on < 0) {
            const char* e = std::getenv("FH_SPMM2");
            on = e ? (std::atoi(e) != 0) : 1;
        }
        if (on && m % 2 == 0 && m >= 16 && m <= 512 && spmm_colblock(m / 2) >= 8 && A.maxrow >= 1 && A.maxrow <= 5) {
            spmm_rows2_launch<TA, CONJ, 5, 2>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out);
            return true;
        }
    }
    // column blocks of at least 16 columns: at most 16 row groups per block
    if (m < 16 || m > 256 || A.maxrow < 1) return false;
    if (A.maxrow <= 5) spmm_rows_launch<T, TA, CONJ, 5, 4>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out);
    else if (A.maxrow <= 8) spmm_rows_launch<T, TA, CONJ, 8, 4>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out);
    else if (A.maxrow <= 16) spmm_rows_launch<T, TA, CONJ, 16, 2>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out);
    else if (A.maxrow <= 32) spmm_rows_launch<T, TA, CONJ, 32, 1>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out);
    else return false;
    return true;
}

template <typename T>
void spmm(hipStream_t st, const CsrDev& A, bool conj_t, int n, int m, int nsys, const Cx<T>* shifts, T alpha,
          const Cx<T>* X, const Cx<T>* Yadd, Cx<T>* Out) {
    if (nsys <= 0) return;
    const int ry = m >= 256 ? 1 : std::max(1, 256 / m);
    dim3 blk(m, ry), grid(ceil_div(n, ry), nsys);
    hipEvent_t ev = prof_begin(st);
    if (A.complex_vals) {
        const Cx<T>* v = (const Cx<T>*)A.val<T>();
        if (conj_t) {
            if (!spmm_rows<T, Cx<T>, true>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out))
                k_spmm<T, Cx<T>, true><<<grid, blk, 0, st>>>(n, m, A.rowptr, A.col, v, shifts, alpha, X, Yadd, Out);
        } else {
            if (!spmm_rows<T, Cx<T>, false>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out))
                k_spmm<T, Cx<T>, false><<<grid, blk, 0, st>>>(n, m, A.rowptr, A.col, v, shifts, alpha, X, Yadd, Out);
        }
    } else {
        const T* v = (const T*)A.val<T>();
        if (!spmm_rows<T, T, false>(st, n, m, nsys, A, v, shifts, alpha, X, Yadd, Out))
            k_spmm<T, T, false><<<grid, blk, 0, st>>>(n, m, A.rowptr, A.col, v, shifts, alpha, X, Yadd, Out);
    }
    FH_LAUNCH_CHECK();
    if (ev) {
        // algorithmic bytes: X in, Out (and Yadd) once each, the CSR arrays once
        const double vec = (double)nsys * n * m * sizeof(Cx<T>);
        const double mat = (double)A.nnz * ((A.complex_vals ? 2 : 1) * sizeof(T) + 4) + 4.0 * (n + 1);
        prof_end(st, ev, std::string("spmm_") + (sizeof(T) == 8 ? "c128" : "c64"), vec * (Yadd ? 3 : 2) + mat,
                 (double)nsys * m * (8.0 * A.nnz + 8.0 * n));
    }
}
template void spmm<double>(hipStream_t, const CsrDev&, bool, int, int, int, const zd*, double, const zd*, const zd*, zd*);
template void spmm<float>(hipStream_t, const CsrDev&, bool, int, int, int, const cf*, float, const cf*, const cf*, cf*);

// ---------------------------------------------------------------------------
// M_j values on the pattern of M = A + diag: z_j on the diagonal minus A
// ---------------------------------------------------------------------------
__global__ void k_zero(long len, zd* __restrict__ p) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) p[e] = czero<double>();
}
template <typename TA>
__global__ void k_scatter_negA(long nnzA, long nnzM, const TA* __restrict__ Aval, const int* __restrict__ a2m,
                               zd* __restrict__ out) {
    const int j = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnzA) return;
    zd v;
    if constexpr (sizeof(TA) == sizeof(double)) v = cx(-(double)Aval[e], 0.0);
    else v = -Aval[e];
    out[(long)j * nnzM + a2m[e]] = v;
}
__global__ void k_add_diag(int n, long nnzM, const int* __restrict__ diag, const zd* __restrict__ z, zd* __restrict__ out) {
    const int j = blockIdx.y;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    zd* o = out + (long)j * nnzM + diag[i];
    *o = *o + z[j];
}

void form_mvals(hipStream_t st, const SparseState& S, int ne, const zd* z_dev, zd* out) {
    const long nnzM = S.nnzM;
    dim3 g1(ceil_div(nnzM * ne, 256));
    k_zero<<<g1, 256, 0, st>>>(nnzM * ne, out);
    FH_LAUNCH_CHECK();
    dim3 g2(ceil_div(S.nnzA, 256), ne);
    if (S.A.complex_vals) k_scatter_negA<zd><<<g2, 256, 0, st>>>(S.nnzA, nnzM, (const zd*)S.A.val64, S.a2m, out);
    else k_scatter_negA<double><<<g2, 256, 0, st>>>(S.nnzA, nnzM, (const double*)S.A.val64, S.a2m, out);
    FH_LAUNCH_CHECK();
    dim3 g3(ceil_div(S.n, 256), ne);
    k_add_diag<<<g3, 256, 0, st>>>(S.n, nnzM, S.mdiag, z_dev, out);
    FH_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// ILU(0) numeric factorization, one workgroup per node, rows by level
// (IKJ order within a row: L entries in increasing column order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ilu0_factor(int n, long nnzM, const int* __restrict__ rowptr,
                                                     const int* __restrict__ col, const int* __restrict__ diag,
                                                     const int* __restrict__ uptr, const int2* __restrict__ upd,
                                                     const int* __restrict__ lev_ptr, const int* __restrict__ lev_rows,
                                                     int nlev, zd* __restrict__ lu_all) {
    zd* lu = lu_all + (long)blockIdx.x * nnzM;
    for (int lev = 0; lev < nlev; ++lev) {
        const int t1 = lev_ptr[lev + 1];
        for (int t = lev_ptr[lev] + threadIdx.x; t < t1; t += blockDim.x) {
            const int i = lev_rows[t];
            const int pd = diag[i];
            for (int p = rowptr[i]; p < pd; ++p) {
                const int k = col[p];
                const zd l = cdiv(lu[p], lu[diag[k]]);
                lu[p] = l;
                const int u1 = uptr[p + 1];
                for (int u = uptr[p]; u < u1; ++u) {
                    const int2 q = upd[u];
                    cfms(lu[q.x], l, lu[q.y]);
                }
            }
        }
        __syncthreads();
    }
}

// luT[q] = lu[t2m[q]];  dinv[i] = 1 / u_ii  (per node)
__global__ void k_ilu0_post(int n, long nnzM, const int* __restrict__ t2m, const int* __restrict__ diag,
                            const zd* __restrict__ lu_all, zd* __restrict__ luT_all, zd* __restrict__ dinv_all) {
    const int j = blockIdx.y;
    const zd* lu = lu_all + (long)j * nnzM;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnzM) luT_all[(long)j * nnzM + e] = lu[t2m[e]];
    if (e < n) dinv_all[(long)j * n + e] = cdiv(cx(1.0, 0.0), lu[diag[e]]);
}

template <typename D>
__global__ void k_cast_d(long len, const zd* __restrict__ s, Cx<D>* __restrict__ d) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) d[e] = ccast<D>(s[e]);
}

void ilu0_factor(hipStream_t st, const SparseState& S, int ne, zd* lu, zd* luT, zd* dinv) {
    k_ilu0_factor<<<ne, 256, 0, st>>>(S.n, S.nnzM, S.mrowptr, S.mcol, S.mdiag, S.uptr, S.upd, S.levL.ptr,
                                      S.levL.rows, S.levL.nlev, lu);
    FH_LAUNCH_CHECK();
    dim3 g(ceil_div(std::max<long>(S.nnzM, S.n), 256), ne);
    k_ilu0_post<<<g, 256, 0, st>>>(S.n, S.nnzM, S.t2m, S.mdiag, lu, luT, dinv);
    FH_LAUNCH_CHECK();
}

void to_single(hipStream_t st, long len, const zd* s, cf* d) {
    if (len <= 0) return;
    k_cast_d<float><<<ceil_div(len, 256), 256, 0, st>>>(len, s, d);
    FH_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Packing of the factor values into the level-packed ELL order of a sweep
// (per node), conjugated for the left-side sweeps; pivots inverted.
// ---------------------------------------------------------------------------
__global__ void k_pack_ell(int n, int K, const int* __restrict__ pos, const zd* __restrict__ lu_all, long nnzM,
                           int conjv, zd* __restrict__ out_all) {
    const int j = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)K * n) return;
    const int p = pos[e];
    zd v = p >= 0 ? lu_all[(long)j * nnzM + p] : czero<double>();
    out_all[(long)j * K * n + e] = conjv ? conj(v) : v;
}
__global__ void k_pack_diag(int n, const int* __restrict__ dpos, const zd* __restrict__ lu_all, long nnzM, int conjv,
                            zd* __restrict__ out_all) {
    const int j = blockIdx.y;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    zd v = cdiv(cx(1.0, 0.0), lu_all[(long)j * nnzM + dpos[t]]);
    out_all[(long)j * n + t] = conjv ? conj(v) : v;
}
void pack_sweep_vals(hipStream_t st, const SweepDev& sw, int n, int ne, long nnzM, const zd* lu, zd* ell, zd* diag) {
    if (sw.K > 0) {
        dim3 g(ceil_div((size_t)sw.K * n, 256), ne);
        k_pack_ell<<<g, 256, 0, st>>>(n, sw.K, sw.ell_pos, lu, nnzM, sw.conj ? 1 : 0, ell);
        FH_LAUNCH_CHECK();
    }
    if (sw.dpos && diag) {
        dim3 g(ceil_div(n, 256), ne);
        k_pack_diag<<<g, 256, 0, st>>>(n, sw.dpos, lu, nnzM, sw.conj ? 1 : 0, diag);
        FH_LAUNCH_CHECK();
    }
}

// ---------------------------------------------------------------------------
// Preconditioner apply: Out_s = (L U)^{-1} X_s (side 0) or (L U)^{-H} X_s
// (side 1) with the factors of node(s).  One workgroup per (column chunk,
// system) sweeps the rows level by level; within a level each thread first
// issues the loads of up to P items (independent of the level's stores), then
// stores them.
// ---------------------------------------------------------------------------
// everything an item needs that does not depend on the sweep's own results:
// its row, column, ELL slot, dependency columns, input value, and the factor
// values and pivot (all prefetched one level ahead, so only the loads of the
// previous levels' results are waited on inside a level)
template <typename T, int KM>
struct SwItem {
    int row, cc;
    int col[KM];
    Cx<T> xin, d;
    Cx<T> v[KM];
};

template <typename T, int P, int KM>
__device__ __forceinline__ void load_items(const SweepDev& sw, int n, int m, int c0, int cw, const Cx<T>* __restrict__ val,
                                           const Cx<T>* __restrict__ dval, const Cx<T>* In, int lev, int base,
                                           SwItem<T, KM>* it) {
    const int t0 = sw.lev_ptr[lev];
    const int items = (sw.lev_ptr[lev + 1] - t0) * cw;
    const int K = sw.K;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e = base + threadIdx.x + 256 * q;
        it[q].row = -1;
        if (e < items) {
            const int t = t0 + e / cw;
            const int cc = c0 + e % cw;
            const int row = sw.rows[t];
            it[q].row = row;
            it[q].cc = cc;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const bool on = k < K;
                it[q].col[k] = on ? sw.ell_col[(long)k * n + t] : -1;
                it[q].v[k] = on ? val[(long)k * n + t] : czero<T>();
            }
            it[q].d = dval ? dval[t] : cx(T(1), T(0));
            it[q].xin = In[(long)row * m + cc];
        }
    }
}

// loads of the previous levels' results for all items first, then the
// caller's prefetch of the next level, then the stores
template <typename T, int P, int KM, typename Between>
__device__ __forceinline__ void solve_items(const SwItem<T, KM>* it, int n, int m, Cx<T>* Os, Between between) {
    Cx<T> xs[P][KM];
#pragma unroll
    for (int q = 0; q < P; ++q) {
#pragma unroll
        for (int k = 0; k < KM; ++k) xs[q][k] = czero<T>();
        if (it[q].row >= 0) {
#pragma unroll
            for (int k = 0; k < KM; ++k)
                if (it[q].col[k] >= 0) xs[q][k] = Os[(long)it[q].col[k] * m + it[q].cc];
        }
    }
    between();
#pragma unroll
    for (int q = 0; q < P; ++q) {
        if (it[q].row >= 0) {
            Cx<T> v = it[q].xin;
#pragma unroll
            for (int k = 0; k < KM; ++k) cfms(v, it[q].v[k], xs[q][k]);
            Os[(long)it[q].row * m + it[q].cc] = it[q].d * v;
        }
    }
}

template <typename T, int P, int KM>
__device__ __forceinline__ void sweep(const SweepDev& sw, int n, int m, int c0, int cw, const Cx<T>* __restrict__ val,
                                      const Cx<T>* __restrict__ dval, const Cx<T>* In, Cx<T>* Os) {
    if (sw.nlev <= 0) return;
    SwItem<T, KM> cur[P], nxt[P];
    load_items<T, P, KM>(sw, n, m, c0, cw, val, dval, In, 0, 0, cur);
    for (int lev = 0; lev < sw.nlev; ++lev) {
        // the current level's loads are issued first, then the prefetch of the
        // next level's independent data, so waiting on the former does not
        // wait on the latter (loads retire in issue order)
        solve_items<T, P, KM>(cur, n, m, Os, [&] {
            if (lev + 1 < sw.nlev) load_items<T, P, KM>(sw, n, m, c0, cw, val, dval, In, lev + 1, 0, nxt);
        });
        const int items = (sw.lev_ptr[lev + 1] - sw.lev_ptr[lev]) * cw;
        for (int base = 256 * P; base < items; base += 256 * P) {     // levels wider than one batch
            SwItem<T, KM> tmp[P];
            load_items<T, P, KM>(sw, n, m, c0, cw, val, dval, In, lev, base, tmp);
            solve_items<T, P, KM>(tmp, n, m, Os, [] {});
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) cur[q] = nxt[q];
    }
}

// Deeper pipeline for narrow sweeps (KM <= 4): the level pointers are read
// three levels ahead, the t-indexed data (row, dependency columns, factor
// values, pivot) two levels ahead, the input value (which needs the row) one
// level ahead, so that inside a level only the loads of the previous levels'
// results are waited on and no chain of dependent memory loads remains.
template <typename T, int KM>
struct SwA {
    int row, cc;
    int col[KM];
    Cx<T> v[KM];
    Cx<T> d;
};

template <typename T, int P, int KM>
__device__ __forceinline__ void load_a(const SweepDev& sw, int n, int c0, int cw, const Cx<T>* __restrict__ val,
                                       const Cx<T>* __restrict__ dval, int t0, int t1, SwA<T, KM>* a) {
    const int items = (t1 - t0) * cw;
    const int K = sw.K;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e = threadIdx.x + 256 * q;
        a[q].row = -1;
        if (e < items) {
            const int t = t0 + e / cw;
            a[q].row = sw.rows[t];
            a[q].cc = c0 + e % cw;
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const bool on = k < K;
                a[q].col[k] = on ? sw.ell_col[(long)k * n + t] : -1;
                a[q].v[k] = on ? val[(long)k * n + t] : czero<T>();
            }
            a[q].d = dval ? dval[t] : cx(T(1), T(0));
        }
    }
}

template <typename T, int P, int KM>
__device__ __forceinline__ void sweep_deep(const SweepDev& sw, int n, int m, int c0, int cw,
                                           const Cx<T>* __restrict__ val, const Cx<T>* __restrict__ dval,
                                           const Cx<T>* In, Cx<T>* Os) {
    const int nlev = sw.nlev;
    if (nlev <= 0) return;
    auto LP = [&](int l) { return sw.lev_ptr[l <= nlev ? l : nlev]; };
    int p0 = LP(0), p1 = LP(1), p2 = LP(2), p3 = LP(3);
    SwA<T, KM> a0[P], a1[P], a2[P];
    Cx<T> x0[P], x1[P];
    load_a<T, P, KM>(sw, n, c0, cw, val, dval, p0, p1, a0);
    load_a<T, P, KM>(sw, n, c0, cw, val, dval, p1, p2, a1);
#pragma unroll
    for (int q = 0; q < P; ++q) x0[q] = a0[q].row >= 0 ? In[(long)a0[q].row * m + a0[q].cc] : czero<T>();
    for (int lev = 0; lev < nlev; ++lev) {
        const int p4 = LP(lev + 4);
        // results of the previous levels this level depends on
        Cx<T> xs[P][KM];
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int k = 0; k < KM; ++k)
                xs[q][k] = (a0[q].row >= 0 && a0[q].col[k] >= 0) ? Os[(long)a0[q].col[k] * m + a0[q].cc]
                                                                 : czero<T>();
        // prefetch: inputs of level lev+1, t-indexed data of level lev+2
#pragma unroll
        for (int q = 0; q < P; ++q)
            x1[q] = (lev + 1 < nlev && a1[q].row >= 0) ? In[(long)a1[q].row * m + a1[q].cc] : czero<T>();
        if (lev + 2 < nlev) load_a<T, P, KM>(sw, n, c0, cw, val, dval, p2, p3, a2);
#pragma unroll
        for (int q = 0; q < P; ++q) {
            if (a0[q].row >= 0) {
                Cx<T> v = x0[q];
#pragma unroll
                for (int k = 0; k < KM; ++k) cfms(v, a0[q].v[k], xs[q][k]);
                Os[(long)a0[q].row * m + a0[q].cc] = a0[q].d * v;
            }
        }
        const int items = (p1 - p0) * cw;
        for (int base = 256 * P; base < items; base += 256 * P) {     // levels wider than one batch
            SwItem<T, KM> tmp[P];
            load_items<T, P, KM>(sw, n, m, c0, cw, val, dval, In, lev, base, tmp);
            solve_items<T, P, KM>(tmp, n, m, Os, [] {});
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < P; ++q) {
            a0[q] = a1[q];
            a1[q] = a2[q];
            x0[q] = x1[q];
        }
        p0 = p1;
        p1 = p2;
        p2 = p3;
        p3 = p4;
    }
}

// Sweep whose dependencies all lie in the previous level (true for the
// natural-order ILU(0) of a 5-point stencil: anti-diagonal levels): the last
// two levels' results for the workgroup's columns live in an LDS ring, so a
// level waits only on LDS and its barrier on LDS traffic; the results still
// go to global memory, which nothing inside the sweep reads back.
template <typename T, int KM>
struct SwL {
    int row, cc, pos;
    bool act;
    int slot[KM];
    Cx<T> v[KM];
    Cx<T> d;
};

// Prefetch of the t-indexed data of a level.  Branch-free and without any
// arithmetic on the loaded values (which would make the compiler wait for
// them here): every load uses a clamped, valid index; masks are applied
// where the values are used.
template <typename T, int P, int KM, int NT>
__device__ __forceinline__ void load_l(const SweepDev& sw, int n, int c0, int cw, const Cx<T>* __restrict__ val,
                                       const Cx<T>* __restrict__ dval, int t0, int t1, int base, SwL<T, KM>* a) {
    const int items = (t1 - t0) * cw;
    const int K = sw.K;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e0 = base + threadIdx.x + NT * q;
        const bool act = e0 < items;
        const int e = act ? e0 : 0;
        const int t = min(t0 + e / cw, n - 1);      // t0 may be n past the last level
        a[q].row = sw.rows[t];
        a[q].act = act;
        a[q].cc = e % cw;
        a[q].pos = t - t0;
        if (K > 0) {                                 // uniform
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int kk = k < K ? k : 0;
                a[q].slot[k] = sw.ell_slot[(long)kk * n + t];
                a[q].v[k] = val[(long)kk * n + t];
            }
        }
        a[q].d = dval ? dval[t] : cx(T(1), T(0));
    }
}

// wait for this workgroup's LDS traffic only, then barrier
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

template <typename T, int P, int KM, int NT>
__device__ __forceinline__ void sweep_lds(const SweepDev& sw, int n, int m, int c0, int cw,
                                          const Cx<T>* __restrict__ val, const Cx<T>* __restrict__ dval,
                                          const Cx<T>* In, Cx<T>* Os, Cx<T>* ring, int ring_stride) {
    const int nlev = sw.nlev;
    if (nlev <= 0) return;
    auto LP = [&](int l) { return sw.lev_ptr[l <= nlev ? l : nlev]; };
    int p0 = LP(0), p1 = LP(1), p2 = LP(2), p3 = LP(3);
    SwL<T, KM> a0[P], a1[P], a2[P];
    Cx<T> x0[P], x1[P];
    load_l<T, P, KM, NT>(sw, n, c0, cw, val, dval, p0, p1, 0, a0);
    load_l<T, P, KM, NT>(sw, n, c0, cw, val, dval, p1, p2, 0, a1);
#pragma unroll
    for (int q = 0; q < P; ++q) x0[q] = In[(long)a0[q].row * m + c0 + a0[q].cc];
    for (int lev = 0; lev < nlev; ++lev) {
        const int p4 = LP(lev + 4);
        const Cx<T>* prev = ring + (long)((lev + 1) & 1) * ring_stride;
        Cx<T>* cur = ring + (long)(lev & 1) * ring_stride;
        // prefetch: inputs of level lev+1, t-indexed data of level lev+2
#pragma unroll
        for (int q = 0; q < P; ++q) x1[q] = In[(long)a1[q].row * m + c0 + a1[q].cc];
        load_l<T, P, KM, NT>(sw, n, c0, cw, val, dval, p2, p3, 0, a2);
        const int items = (p1 - p0) * cw;
        for (int base = 0; base < items; base += NT * P) {
            SwL<T, KM> b[P];
            Cx<T> xb[P];
            if (base == 0) {
#pragma unroll
                for (int q = 0; q < P; ++q) { b[q] = a0[q]; xb[q] = x0[q]; }
            } else {                                   // levels wider than one batch
                load_l<T, P, KM, NT>(sw, n, c0, cw, val, dval, p0, p1, base, b);
#pragma unroll
                for (int q = 0; q < P; ++q) xb[q] = In[(long)b[q].row * m + c0 + b[q].cc];
            }
#pragma unroll
            for (int q = 0; q < P; ++q) {
                if (b[q].act) {
                    Cx<T> v = xb[q];
#pragma unroll
                    for (int k = 0; k < KM; ++k) {
                        const int sl = b[q].slot[k];
                        if (k < sw.K && sl >= 0) cfms(v, b[q].v[k], prev[sl * cw + b[q].cc]);
                    }
                    v = b[q].d * v;
                    cur[b[q].pos * cw + b[q].cc] = v;
                    Os[(long)b[q].row * m + c0 + b[q].cc] = v;
                }
            }
        }
        lds_barrier();
#pragma unroll
        for (int q = 0; q < P; ++q) {
            a0[q] = a1[q];
            a1[q] = a2[q];
            x0[q] = x1[q];
        }
        p0 = p1;
        p1 = p2;
        p2 = p3;
        p3 = p4;
    }
}

// Sweep with a deeper prefetch for levels that fit one batch (at most NT
// rows and P * NT / cw items per level, at least one off-diagonal slot per
// sweep).  A level's time is the latency it waits for, so every load a level
// uses is issued three levels earlier, the row indices (on which the input
// addresses depend) six levels earlier.  The factor data of a row (its
// dependency slots, values and pivot) are loaded once per row, by the thread
// of that row, and passed to the level's other threads through a two-level
// LDS ring: per thread one row's worth of registers instead of one per item,
// which keeps the four prefetch slots within the register file.  Nothing in
// the loop branches on a thread's data (the compiler then counts the loads in
// flight exactly):
//  * the loop is unrolled by four, so each slot keeps its registers;
//  * prefetches past the last level repeat the last level (in bounds, unused);
//  * a thread whose item (or row) lies past the end of a narrower level
//    repeats the level's last one: same inputs, same value, same address;
//  * absent dependencies (slot < 0) contribute a selected zero;
//  * the level pointers are read through the scalar cache.
template <typename T, int P, int KM, int FR>
struct SwPipe {
    int row[P];          // row indices of a level (loaded six levels ahead)
    Cx<T> x[P];          // inputs of a level (three levels ahead)
    int off[P];          // element offsets of those inputs / outputs
    int fslot[FR][KM];   // factor data of FR rows (four levels ahead)
    Cx<T> fv[FR][KM];
    Cx<T> fd[FR];
};

// FR: level rows whose factor data each thread loads (levels of up to NT * FR rows)
template <typename T, int P, int KM, int NT, int FR>
__device__ __forceinline__ void sweep_pipe(const SweepDev& sw, int n, int m, int c0, int cw,
                                           const Cx<T>* __restrict__ val, const Cx<T>* __restrict__ dval,
                                           const Cx<T>* In, Cx<T>* Os, Cx<T>* ring, int ring_stride,
                                           int* fslot_l, Cx<T>* fv_l, Cx<T>* fd_l, int wmax, Cx<T>* junk) {
    static_assert(NT * P <= ILU_JUNK, "junk buffer too small for one level's items");
    const int nlev = sw.nlev;
    if (nlev <= 0) return;
    using CI = const __attribute__((address_space(4))) int;
    CI* lp = (CI*)sw.lev_ptr;
    const int K = sw.K;
    const bool hasd = dval != nullptr;
    const Cx<T>* dsrc = hasd ? dval : val;         // unit sweeps load (and ignore) a valid entry
    const int tid = threadIdx.x;
    int ediv[P], emod[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e0 = tid + NT * q;
        ediv[q] = e0 / cw;
        emod[q] = e0 % cw;
    }
    // level position of item q (or, for q < 0, of this thread's row) of level l, clamped
    auto pos_of = [&](int l, int r) {
        const int L = min(max(l, 0), nlev - 1);
        const int t0 = lp[L], rows = lp[L + 1] - t0;
        return min(t0 + min(r, rows - 1), n - 1);
    };
    using SP = SwPipe<T, P, KM, FR>;
    auto load_row = [&](int l, SP& s) {
#pragma unroll
        for (int q = 0; q < P; ++q) s.row[q] = sw.rows[pos_of(l, ediv[q])];
    };
    auto load_x = [&](SP& s) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            s.off[q] = (int)__umul24((unsigned)s.row[q], (unsigned)m) + c0 + emod[q];   // as in sweep_vec
            s.x[q] = In[s.off[q]];
        }
    };
    auto load_fac = [&](int l, SP& s) {
#pragma unroll
        for (int f = 0; f < FR; ++f) {
            const int t = pos_of(l, tid + f * NT);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int kk = k < K ? k : 0;
                s.fslot[f][k] = sw.ell_slot[(long)kk * n + t];
                s.fv[f][k] = val[(long)kk * n + t];
            }
            s.fd[f] = dsrc[t];
        }
    };
    // factor data of one level into LDS ring slot b (rows past the level's end repeat its last row)
    auto put_fac = [&](const SP& s, int b) {
#pragma unroll
        for (int f = 0; f < FR; ++f) {
            const int r = tid + f * NT;
            if (r < wmax) {
#pragma unroll
                for (int k = 0; k < KM; ++k) {
                    fslot_l[(b * wmax + r) * KM + k] = s.fslot[f][k];
                    fv_l[(b * wmax + r) * KM + k] = s.fv[f][k];
                }
                fd_l[b * wmax + r] = s.fd[f];
            }
        }
    };
    // Slot of level L: L mod 4 for each kind of data (row indices live from
    // level L-6 to L-3, inputs from L-3 to L, factor data from L-4 to L-1).
    // At level l, with a, b, c, d the slots of l .. l+3: inputs of level l+3
    // (rows in d), factor data of level l+1 (in b) to LDS, rows of level l+6
    // (slot c), factor data of level l+4 (slot a), then level l from a and
    // LDS.  Every wait is for loads issued three levels earlier.
    auto level = [&](int l, SP& a, SP& b, SP& c, SP& d) {
        load_x(d);
        put_fac(b, (l + 1) & 1);
        load_row(l + 6, c);
        load_fac(l + 4, a);
        const int Lc = max(l, 0);
        const int rows = lp[Lc + 1] - lp[Lc];
        const Cx<T>* prev = ring + (long)((l + 1) & 1) * ring_stride;
        Cx<T>* cur = ring + (long)(l & 1) * ring_stride;
        const int fb = (l & 1) * wmax;
        const bool real = l >= 0 && l < nlev;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int pos = min(ediv[q], rows - 1);
            Cx<T> v = a.x[q];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const int sl = fslot_l[(fb + pos) * KM + k];
                const bool dep = k < K && sl >= 0;
                const Cx<T> pv = prev[(dep ? sl : 0) * cw + emod[q]];
                cfms(v, fv_l[(fb + pos) * KM + k], dep ? pv : czero<T>());
            }
            if (hasd) v = fd_l[fb + pos] * v;
            cur[pos * cw + emod[q]] = v;
            // fill and drain levels write to the junk buffer (a select, not a branch)
            Cx<T>* dst = real ? Os + a.off[q] : junk + (tid + NT * q);
            *dst = v;
        }
        lds_barrier();
    };
    // One loop, one exit: the loop starts at level -8, and its first eight
    // levels only fill the pipeline (their loads repeat level 0's rows, their
    // results go to the junk buffer, and the factor data they read from LDS is
    // the "no dependency" record written here); up to three drain levels past
    // the last repeat its rows in the same way.  The compiler inserts its
    // waits for loads in flight by merging every path into the loop header:
    // a prologue of its own, or a break after each unrolled level, would merge
    // histories with fewer loads issued since and make the header wait for
    // loads of the previous level.
    auto blank = [&](SP& sp) {
#pragma unroll
        for (int q = 0; q < P; ++q) sp.row[q] = 0;
#pragma unroll
        for (int f = 0; f < FR; ++f) {
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                sp.fslot[f][k] = -1;
                sp.fv[f][k] = czero<T>();
            }
            sp.fd[f] = czero<T>();
        }
    };
    SP s0, s1, s2, s3;
    blank(s0);
    blank(s1);
    blank(s2);
    blank(s3);
    for (int i = tid; i < 2 * wmax; i += NT) {
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            fslot_l[i * KM + k] = -1;
            fv_l[i * KM + k] = czero<T>();
        }
        fd_l[i] = czero<T>();
    }
    __syncthreads();
    for (int l = -8; l < nlev; l += 4) {
        level(l, s0, s1, s2, s3);
        level(l + 1, s1, s2, s3, s0);
        level(l + 2, s2, s3, s0, s1);
        level(l + 3, s3, s0, s1, s2);
    }
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.  The
// column blocks of one system share the factor data, and neighbouring blocks
// share the 128-byte lines of the vectors: this mapping gives consecutive
// blocks of a system consecutive workgroups of the same XCD.  Returns the
// (system, column block) of this workgroup.
__device__ __forceinline__ int2 xcd_block() {
    int lin = blockIdx.x + blockIdx.y * gridDim.x;
    const int G = gridDim.x * gridDim.y;
    if (G % 8 == 0) lin = (lin % 8) * (G / 8) + lin / 8;
    return make_int2(lin / gridDim.x, lin % gridDim.x);
}

template <typename T, int P, int KM, int NT, int FR>
__global__ __launch_bounds__(NT) void k_ilu_apply_pipe(IluApplyArgs<T> a, const Cx<T>* __restrict__ X, Cx<T>* Out,
                                                       int ring_stride, int wmax) {
    extern __shared__ unsigned char dsm[];
    Cx<T>* ring = reinterpret_cast<Cx<T>*>(dsm);                 // [2][wmax][cw]
    Cx<T>* fv_l = ring + 2 * ring_stride;                         // [2][wmax][KM]
    Cx<T>* fd_l = fv_l + 2 * wmax * KM;                           // [2][wmax]
    int* fslot_l = reinterpret_cast<int*>(fd_l + 2 * wmax);       // [2][wmax][KM]
    const int2 sb = xcd_block();
    const int s = sb.x;
    const int c0 = sb.y * a.cw;
    const int cw = min(a.cw, a.m - c0);
    const int node = a.node_of[s], side = a.side_of[s];
    const long base = (long)s * a.n * a.m;
    const SweepDev& F = a.fwd[side];
    const SweepDev& B = a.bwd[side];
    const Cx<T>* fv = a.fval[side] + (long)node * F.K * a.n;
    const Cx<T>* fd = a.fdiag[side] ? a.fdiag[side] + (long)node * a.n : nullptr;
    const Cx<T>* bv = a.bval[side] + (long)node * B.K * a.n;
    const Cx<T>* bd = a.bdiag[side] ? a.bdiag[side] + (long)node * a.n : nullptr;
    sweep_pipe<T, P, KM, NT, FR>(F, a.n, a.m, c0, cw, fv, fd, X + base, Out + base, ring, ring_stride, fslot_l, fv_l,
                                 fd_l, wmax, a.junk);
    // the backward sweep starts with the rows other waves stored last in the
    // forward sweep, whose stores the sweep loop leaves in flight
    __threadfence();
    __syncthreads();
    sweep_pipe<T, P, KM, NT, FR>(B, a.n, a.m, c0, cw, bv, bd, Out + base, Out + base, ring, ring_stride, fslot_l, fv_l,
                                 fd_l, wmax, a.junk);
}

// Complex-FP32 sweep with two columns per lane.  A lane owns P items of a
// level, each two adjacent columns of one row (one 16-byte load and store);
// the lanes of a row (cw / 2 of them) each load that row's factor data into
// their own registers, four levels ahead, so no factor data passes through
// LDS: per item and level the LDS traffic is the KM dependency reads from the
// previous level's ring and one write.  Same pipeline as sweep_pipe (row
// indices six levels ahead, inputs three, factor data issued after the
// level's own use of its slot), one loop with fill and drain levels.
__device__ __forceinline__ void c2_fms(float4& acc, float2 a, float4 b) {   // acc -= a * b (both columns)
    acc.x = fmaf(-a.x, b.x, fmaf(a.y, b.y, acc.x));
    acc.y = fmaf(-a.x, b.y, fmaf(-a.y, b.x, acc.y));
    acc.z = fmaf(-a.x, b.z, fmaf(a.y, b.w, acc.z));
    acc.w = fmaf(-a.x, b.w, fmaf(-a.y, b.z, acc.w));
}
__device__ __forceinline__ float4 c2_mul(float2 a, float4 b) {
    return make_float4(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x, a.x * b.z - a.y * b.w, a.x * b.w + a.y * b.z);
}

template <int P, int KM>
struct SwVec {
    int row[P];           // row indices (six levels ahead)
    int pos[P];           // their positions in the packed level order (for the factor data)
    float4 x[P];          // inputs (three levels ahead)
    unsigned off[P];      // byte offsets of those inputs / outputs
    int fslot[P][KM];     // factor data of the items' rows (four levels ahead)
    float2 fv[P][KM];
    float2 fd[P];
};

// loads and stores by a uniform base and a 32-bit byte offset (the address
// form with the base in scalar registers: no 64-bit address arithmetic per lane)
template <typename V>
__device__ __forceinline__ V ld_at(const void* base, unsigned off) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + off);
}
template <typename V>
__device__ __forceinline__ void st_at(void* base, unsigned off, V v) {
    *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + off) = v;
}

// BLK: In / Os in the blocked layout (the workgroup's column block of every
// row contiguous, rows in the forward L sweep's packed order: a level's rows
// are one contiguous run); else the natural layout [row][m]
template <int P, int KM, int NT, int LPR, bool BLK>
__device__ __forceinline__ void sweep_vec(const SweepDev& sw, int n, int m2, int c02,
                                          const float2* __restrict__ val, const float2* __restrict__ dval,
                                          const float4* In, float4* Os, float4* ring, int ring_stride, float4* junk) {
    static_assert(NT * P <= ILU_JUNK / 2, "junk buffer too small for one level's items");
    const int nlev = sw.nlev;
    if (nlev <= 0) return;
    using CI = const __attribute__((address_space(4))) int;
    CI* lp = (CI*)sw.lev_ptr;
    const int K = sw.K;
    const bool hasd = dval != nullptr;
    const float2* dsrc = hasd ? dval : val;
    const int tid = threadIdx.x;
    int ediv[P], emod[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const int e0 = tid + NT * q;
        ediv[q] = e0 / LPR;
        emod[q] = e0 % LPR;
    }
    using SV = SwVec<P, KM>;
    // rows (and packed positions) of level l's items; an item past the end of a
    // narrower level repeats the level's last row; fill and drain levels repeat
    // the first or last level
    auto load_row = [&](int l, SV& s) {
        const int L = min(max(l, 0), nlev - 1);
        const int t0 = lp[L], rows = lp[L + 1] - t0;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            s.pos[q] = min(t0 + min(ediv[q], rows - 1), n - 1);
            s.row[q] = ld_at<int>(BLK ? sw.ppos : sw.rows, (unsigned)s.pos[q] * 4u);
        }
    };
    auto load_x = [&](SV& s) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            // 24-bit multiply: a 32-bit multiply-add becomes a 64-bit one whose
            // unused high addend half the compiler may take from a register a
            // load is still filling, and then it waits for that load
            s.off[q] = BLK ? ((unsigned)s.row[q] * LPR + (unsigned)emod[q]) * 16u
                           : (__umul24((unsigned)s.row[q], (unsigned)m2) + (unsigned)(c02 + emod[q])) * 16u;
            s.x[q] = ld_at<float4>(In, s.off[q]);
        }
    };
    auto load_fac = [&](SV& s) {          // factor data at the positions s.pos
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const unsigned t = (unsigned)s.pos[q];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                const unsigned kk = k < K ? (unsigned)k : 0u;
                const unsigned e = kk * (unsigned)n + t;
                s.fslot[q][k] = ld_at<int>(sw.ell_slot, e * 4u);
                s.fv[q][k] = ld_at<float2>(val, e * 8u);
            }
            s.fd[q] = ld_at<float2>(dsrc, t * 8u);
        }
    };
    const int lw = ring_stride;   // float4 entries of one ring level
    auto level = [&](int l, SV& a, SV& c, SV& d) {
        load_x(d);
        load_row(l + 6, c);
        const int Lc = min(max(l, 0), nlev - 1);
        const int rows = lp[Lc + 1] - lp[Lc];
        const float4* prev = ring + (long)((l + 1) & 1) * lw;
        float4* cur = ring + (long)(l & 1) * lw;
        const bool real = l >= 0 && l < nlev;
        float4* obase = real ? Os : junk;
#pragma unroll
        for (int q = 0; q < P; ++q) {
            const int pos = min(ediv[q], rows - 1);
            float4 v = a.x[q];
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                // an absent dependency reads position 0 with a zero factor (not
                // at load time: the select would wait for the load just issued)
                const bool dep = k < K && a.fslot[q][k] >= 0;
                const float2 f = dep ? a.fv[q][k] : make_float2(0.f, 0.f);
                c2_fms(v, f, prev[(dep ? a.fslot[q][k] : 0) * LPR + emod[q]]);
            }
            if (hasd) v = c2_mul(a.fd[q], v);
            cur[pos * LPR + emod[q]] = v;
            st_at<float4>(obase, real ? a.off[q] : (unsigned)(tid + NT * q) * 16u, v);
        }
        load_fac(a);          // level l + 4: a.pos was set by load_row two levels ago
        lds_barrier();
    };
    auto blank = [&](SV& sv) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
            sv.row[q] = 0;
            sv.pos[q] = 0;
            sv.off[q] = 0;
            sv.x[q] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
                sv.fslot[q][k] = -1;
                sv.fv[q][k] = make_float2(0.f, 0.f);
            }
            sv.fd[q] = make_float2(0.f, 0.f);
        }
    };
    SV s0, s1, s2, s3;
    blank(s0);
    blank(s1);
    blank(s2);
    blank(s3);
    // an absent dependency reads position 0 of the previous level with a zero
    // factor, exact for finite values; the ring starts at zero so that the fill
    // levels (and the first level, which has no dependencies) read finite values
    for (int i = tid; i < 2 * lw; i += NT) ring[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // an opaque start level: with a known one the compiler peels the fill
    // levels into a prologue, which meets the loop header with its own history
    // of loads in flight
    int lstart = -8;
    asm volatile("" : "+s"(lstart));
    for (int l = lstart; l < nlev; l += 4) {
        level(l, s0, s2, s3);
        level(l + 1, s1, s3, s0);
        level(l + 2, s2, s0, s1);
        level(l + 3, s3, s1, s2);
    }
}

// LPR: lanes per row (the workgroup's column block / 2)
// (X and Out may be the same block: the blocked sweep runs in place)
template <int P, int KM, int NT, int LPR, bool BLK>
__global__ __launch_bounds__(NT) void k_ilu_apply_vec(IluApplyArgs<float> a, const Cx<float>* X, Cx<float>* Out,
                                                      int ring_stride) {
    extern __shared__ unsigned char dsm[];
    float4* ring = reinterpret_cast<float4*>(dsm);   // [2][wmax][cw / 2]
    const int2 sb = xcd_block();
    const int s = sb.x;
    const int c0 = sb.y * a.cw;
    const int node = a.node_of[s], side = a.side_of[s];
    // float4 units: the system's block, or (blocked) the system's column block
    const long base = BLK ? ((long)s * (a.m / a.cw) + sb.y) * a.n * LPR : (long)s * a.n * a.m / 2;
    const SweepDev& F = a.fwd[side];
    const SweepDev& B = a.bwd[side];
    const float2* fv = reinterpret_cast<const float2*>(a.fval[side] + (long)node * F.K * a.n);
    const float2* fd = a.fdiag[side] ? reinterpret_cast<const float2*>(a.fdiag[side] + (long)node * a.n) : nullptr;
    const float2* bv = reinterpret_cast<const float2*>(a.bval[side] + (long)node * B.K * a.n);
    const float2* bd = a.bdiag[side] ? reinterpret_cast<const float2*>(a.bdiag[side] + (long)node * a.n) : nullptr;
    const float4* Xv = reinterpret_cast<const float4*>(X) + base;
    float4* Ov = reinterpret_cast<float4*>(Out) + base;
    float4* junk = reinterpret_cast<float4*>(a.junk);
    sweep_vec<P, KM, NT, LPR, BLK>(F, a.n, a.m / 2, c0 / 2, fv, fd, Xv, Ov, ring, ring_stride, junk);
    __threadfence();
    __syncthreads();
    sweep_vec<P, KM, NT, LPR, BLK>(B, a.n, a.m / 2, c0 / 2, bv, bd, Ov, Ov, ring, ring_stride, junk);
}

template <typename T, int P, int KM, int NT>
__global__ __launch_bounds__(NT) void k_ilu_apply_lds(IluApplyArgs<T> a, const Cx<T>* __restrict__ X, Cx<T>* Out,
                                                      int ring_stride) {
    extern __shared__ unsigned char dsm[];
    Cx<T>* ring = reinterpret_cast<Cx<T>*>(dsm);      // [2][wmax][cw]
    const int2 sb = xcd_block();
    const int s = sb.x;
    const int c0 = sb.y * a.cw;
    const int cw = min(a.cw, a.m - c0);
    const int node = a.node_of[s], side = a.side_of[s];
    const long base = (long)s * a.n * a.m;
    const SweepDev& F = a.fwd[side];
    const SweepDev& B = a.bwd[side];
    const Cx<T>* fv = a.fval[side] + (long)node * F.K * a.n;
    const Cx<T>* fd = a.fdiag[side] ? a.fdiag[side] + (long)node * a.n : nullptr;
    const Cx<T>* bv = a.bval[side] + (long)node * B.K * a.n;
    const Cx<T>* bd = a.bdiag[side] ? a.bdiag[side] + (long)node * a.n : nullptr;
    sweep_lds<T, P, KM, NT>(F, a.n, a.m, c0, cw, fv, fd, X + base, Out + base, ring, ring_stride);
    // The backward sweep starts with the rows other waves stored last in the
    // forward sweep: a fence (waits for those stores) before the barrier.
    __threadfence();
    __syncthreads();
    sweep_lds<T, P, KM, NT>(B, a.n, a.m, c0, cw, bv, bd, Out + base, Out + base, ring, ring_stride);
}

template <typename T, int P, int KM>
__global__ __launch_bounds__(256) void k_ilu_apply(IluApplyArgs<T> a, const Cx<T>* __restrict__ X, Cx<T>* Out) {
    const int s = blockIdx.y;
    const int c0 = blockIdx.x * a.cw;
    const int cw = min(a.cw, a.m - c0);
    const int node = a.node_of[s], side = a.side_of[s];
    const long base = (long)s * a.n * a.m;
    const Cx<T>* Xs = X + base;
    Cx<T>* Os = Out + base;
    const SweepDev& F = a.fwd[side];
    const SweepDev& B = a.bwd[side];
    const Cx<T>* fv = a.fval[side] + (long)node * F.K * a.n;
    const Cx<T>* fd = a.fdiag[side] ? a.fdiag[side] + (long)node * a.n : nullptr;
    const Cx<T>* bv = a.bval[side] + (long)node * B.K * a.n;
    const Cx<T>* bd = a.bdiag[side] ? a.bdiag[side] + (long)node * a.n : nullptr;
    if constexpr (KM <= 4) {
        sweep_deep<T, P, KM>(F, a.n, a.m, c0, cw, fv, fd, Xs, Os);
        sweep_deep<T, P, KM>(B, a.n, a.m, c0, cw, bv, bd, Os, Os);
    } else {
        sweep<T, P, KM>(F, a.n, a.m, c0, cw, fv, fd, Xs, Os);
        sweep<T, P, KM>(B, a.n, a.m, c0, cw, bv, bd, Os, Os);
    }
}

// Natural [system][row][m] <-> blocked [system][column block][position][cw]
// layout of complex-FP32 blocks (float4 = two columns; LPR = cw / 2 float4 per
// row and block; position = the row's place in the order `rows`).  A
// workgroup moves BLK_T positions of one system through an LDS tile, so that
// both sides are runs: whole rows on the natural side, BLK_T x LPR float4 per
// column block on the blocked side.  IN: natural -> blocked, else back.
constexpr int BLK_T = 16;
template <bool IN, int TT, int NT>
__global__ __launch_bounds__(NT) void k_blk_perm(int n, int m2, int lpr, const int* __restrict__ rows,
                                                 const float4* __restrict__ src, float4* __restrict__ dst) {
    extern __shared__ unsigned char dsm[];
    float4* tile = reinterpret_cast<float4*>(dsm);   // [TT][m2 + 1]
    const int ld = m2 + 1;
    const int t0 = blockIdx.x * TT, s = blockIdx.y;
    const int nt = min(TT, n - t0);
    const int ncb = m2 / lpr;
    const long nat = (long)s * n * m2;              // system s, natural
    const long blk = (long)s * ncb * n * lpr;       // system s, blocked
    const int tot = nt * m2;
    if (IN) {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int i = e / m2, j = e - i * m2;
            tile[i * ld + j] = src[nat + (long)rows[t0 + i] * m2 + j];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int cb = e / (nt * lpr), r = e - cb * nt * lpr, i = r / lpr, k = r - i * lpr;
            dst[blk + ((long)cb * n + t0 + i) * lpr + k] = tile[i * ld + cb * lpr + k];
        }
    } else {
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int cb = e / (nt * lpr), r = e - cb * nt * lpr, i = r / lpr, k = r - i * lpr;
            tile[i * ld + cb * lpr + k] = src[blk + ((long)cb * n + t0 + i) * lpr + k];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < tot; e += blockDim.x) {
            const int i = e / m2, j = e - i * m2;
            dst[nat + (long)rows[t0 + i] * m2 + j] = tile[i * ld + j];
        }
    }
}
template <int TT, int NT>
static void blk_perm_t(hipStream_t st, bool in, int nsys, int n, int m, int cw, const int* rows, const void* src,
                       void* dst) {
    const int m2 = m / 2;
    dim3 grid(ceil_div(n, TT), nsys);
    const size_t sh = sizeof(float4) * TT * (size_t)(m2 + 1);
    if (in) k_blk_perm<true, TT, NT><<<grid, NT, sh, st>>>(n, m2, cw / 2, rows, (const float4*)src, (float4*)dst);
    else k_blk_perm<false, TT, NT><<<grid, NT, sh, st>>>(n, m2, cw / 2, rows, (const float4*)src, (float4*)dst);
    FH_LAUNCH_CHECK();
}
// tile of 16 rows, 256 threads: measured on one 1024^2 x 160-column block,
// 0.54 + 0.50 ms for the two directions (5.0 / 5.4 TB/s) against 0.80 + 0.67 ms
// with 32 rows and 0.55-0.59 ms with 8 rows or 512 threads
static void blk_perm(hipStream_t st, bool in, int nsys, int n, int m, int cw, const int* rows, const void* src,
                     void* dst) {
    blk_perm_t<BLK_T, 256>(st, in, nsys, n, m, cw, rows, src, dst);
}

// ---------------------------------------------------------------------------
// The operator product after the blocked sweep: Out_s = alpha (sh_s Z_s -
// op(A) Z_s) with Z in the blocked layout [system][column block][position]
// [lpr] and Out natural.  The rows are taken in position order from an ELL
// copy of the operator (SL slots per row: neighbour positions and values,
// empty slots the row itself with weight 0, as in k_spmm_rows2, whose
// arithmetic this repeats entry by entry).  A workgroup takes BLK_T
// consecutive positions of one level and every column: on a level-ordered
// grid the neighbours of a run of positions lie in runs of the levels on
// either side, and the results leave through an LDS tile as whole natural
// rows.  The tiles are dealt to the 8 XCDs by their place within their level
// (workgroup w runs on XCD w mod 8), so that the tiles that read the same
// runs of neighbouring levels share one L2.
// ---------------------------------------------------------------------------
__global__ void k_inv_perm(int n, const int* __restrict__ rows, int* __restrict__ pos) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) pos[rows[t]] = t;
}

template <typename TA>
__global__ void k_blk_ell(int n, const int* __restrict__ rows, const int* __restrict__ pos,
                          const int* __restrict__ rowptr, const int* __restrict__ col, const TA* __restrict__ val,
                          int* __restrict__ bcol, TA* __restrict__ bval) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = rows[t], p0 = rowptr[i], p1 = rowptr[i + 1];
#pragma unroll
    for (int q = 0; q < SPMM_BLK_SL; ++q) {
        const int p = p0 + q;
        const bool has = p < p1;
        bcol[(long)t * SPMM_BLK_SL + q] = has ? pos[col[p]] : t;
        bval[(long)t * SPMM_BLK_SL + q] = has ? val[p] : TA{};
    }
}

template <typename TA, bool CONJ>
__global__ __launch_bounds__(256) void k_spmm_blk(int n, int m2, int lpr, const int2* __restrict__ tiles,
                                                  const int* __restrict__ rows, const int* __restrict__ bcol,
                                                  const TA* __restrict__ bval, const Cx<float>* __restrict__ shifts,
                                                  float alpha, const float4* __restrict__ Z, float4* __restrict__ Out) {
    constexpr int SL = SPMM_BLK_SL;
    extern __shared__ unsigned char dsm[];
    float4* tile = reinterpret_cast<float4*>(dsm);   // [BLK_T][m2 + 1]
    __shared__ int s_col[BLK_T * SL];
    __shared__ TA s_val[BLK_T * SL];
    const int ld = m2 + 1;
    const int2 tl = tiles[blockIdx.x];                // (first position, count <= BLK_T); count 0: padding
    const int t0 = tl.x, nt = tl.y, s = blockIdx.y;
    if (nt <= 0) return;
    const int ncb = m2 / lpr;
    const long nat = (long)s * n * m2;
    const long blk = (long)s * ncb * n * lpr;
    for (int e = threadIdx.x; e < nt * SL; e += blockDim.x) {
        s_col[e] = bcol[(long)t0 * SL + e];
        s_val[e] = bval[(long)t0 * SL + e];
    }
    __syncthreads();
    const Cx<float> sh = shifts[s];
    const int tot = nt * m2;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        const int cb = e / (nt * lpr), r = e - cb * nt * lpr, i = r / lpr, k = r - i * lpr;
        const float4* Zc = Z + blk + (long)cb * n * lpr + k;
        float4 xv[SL];
#pragma unroll
        for (int q = 0; q < SL; ++q) xv[q] = Zc[(long)s_col[i * SL + q] * lpr];
        const float4 xr = Zc[(long)(t0 + i) * lpr];
        Cx<float> a0 = czero<float>(), a1 = czero<float>();
#pragma unroll
        for (int q = 0; q < SL; ++q) {
            mac_val(a0, s_val[i * SL + q], Cx<float>{xv[q].x, xv[q].y}, CONJ);
            mac_val(a1, s_val[i * SL + q], Cx<float>{xv[q].z, xv[q].w}, CONJ);
        }
        Cx<float> r0v = sh * Cx<float>{xr.x, xr.y};
        Cx<float> r1v = sh * Cx<float>{xr.z, xr.w};
        r0v = alpha * (r0v - a0);
        r1v = alpha * (r1v - a1);
        tile[i * ld + cb * lpr + k] = pair_of(r0v, r1v);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
        const int i = e / m2, j = e - i * m2;
        Out[nat + (long)rows[t0 + i] * m2 + j] = tile[i * ld + j];
    }
}

// the ELL copies of A and A^T in position order (once per problem)
static void ensure_blk_ell(hipStream_t st, SparseState& S, const int* order) {
    if (S.bell_ready) return;
    const int n = S.n;
    const bool cv = S.A.complex_vals;
    const size_t vb = cv ? sizeof(cf) : sizeof(float);
    int* pos = (int*)S.bpos.ensure(sizeof(int) * (size_t)n);
    k_inv_perm<<<ceil_div(n, 256), 256, 0, st>>>(n, order, pos);
    FH_LAUNCH_CHECK();
    for (int tr = 0; tr < 2; ++tr) {
        const CsrDev& A = tr ? S.AT : S.A;
        int* bc = (int*)(tr ? S.bcolAT : S.bcolA).ensure(sizeof(int) * (size_t)n * SPMM_BLK_SL);
        void* bv = (tr ? S.bvalAT : S.bvalA).ensure(vb * (size_t)n * SPMM_BLK_SL);
        if (cv)
            k_blk_ell<cf><<<ceil_div(n, 256), 256, 0, st>>>(n, order, pos, A.rowptr, A.col, (const cf*)A.val32, bc,
                                                            (cf*)bv);
        else
            k_blk_ell<float><<<ceil_div(n, 256), 256, 0, st>>>(n, order, pos, A.rowptr, A.col,
                                                               (const float*)A.val32, bc, (float*)bv);
        FH_LAUNCH_CHECK();
    }
    // tiles of at most BLK_T positions within one level; the tiles of a
    // level are split into 8 contiguous groups by their place in it, group x
    // goes to the workgroups w with w mod 8 = x, in level order
    const SweepDev& sw = S.swL;
    std::vector<int> lp(sw.nlev + 1);
    FH_HIP(hipMemcpyAsync(lp.data(), sw.lev_ptr, sizeof(int) * lp.size(), hipMemcpyDeviceToHost, st));
    FH_HIP(hipStreamSynchronize(st));
    std::vector<std::vector<int2>> lists(8);
    for (int l = 0; l < sw.nlev; ++l) {
        const int a = lp[l], b = lp[l + 1], ntl = ceil_div(b - a, BLK_T);
        for (int j = 0; j < ntl; ++j) {
            const int x = (int)((long)j * 8 / ntl);
            const int t0 = a + j * BLK_T;
            lists[x].push_back(int2{t0, std::min(BLK_T, b - t0)});
        }
    }
    size_t len = 0;
    for (const auto& v : lists) len = std::max(len, v.size());
    std::vector<int2> tl(8 * len, int2{0, 0});
    for (int x = 0; x < 8; ++x)
        for (size_t q = 0; q < lists[x].size(); ++q) tl[q * 8 + x] = lists[x][q];
    int2* dt = (int2*)S.btiles.ensure(sizeof(int2) * std::max<size_t>(1, tl.size()));
    FH_HIP(hipMemcpyAsync(dt, tl.data(), sizeof(int2) * tl.size(), hipMemcpyHostToDevice, st));
    FH_HIP(hipStreamSynchronize(st));
    S.btiles_n = (int)tl.size();
    S.bell_ready = true;
}

// the product of `f` from the blocked block P (nsys systems, cw columns per
// block); false when it does not apply (then nothing is launched)
static bool spmm_after_blocked(hipStream_t st, const SpmmAfter& f, int nsys, int n, int m, int cw, const int* order,
                               const cf* P) {
    const char* e = std::getenv("FH_SPMM_BLK");
    if (e && std::atoi(e) == 0) return false;
    const char* e2 = std::getenv("FH_SPMM2");
    if (e2 && std::atoi(e2) == 0) return false;
    SparseState& S = *f.S;
    // the selection of the row-staged two-column product (k_spmm_rows2)
    const bool ok2 = m % 2 == 0 && m >= 16 && m <= 512 && spmm_colblock(m / 2) >= 8;
    const bool okA = S.A.maxrow >= 1 && S.A.maxrow <= SPMM_BLK_SL;
    const bool okT = nsys == f.nright || (S.AT.maxrow >= 1 && S.AT.maxrow <= SPMM_BLK_SL);
    const int m2 = m / 2, lpr = cw / 2;
    const size_t sh = sizeof(float4) * BLK_T * (size_t)(m2 + 1);
    const size_t sh_static = (size_t)BLK_T * SPMM_BLK_SL * (sizeof(int) + sizeof(cf));
    if (!ok2 || !okA || !okT || S.n != n || cw % 2 != 0 || m2 % lpr != 0 || sh + sh_static > 65536) return false;
    ensure_blk_ell(st, S, order);
    const long sysf4 = (long)n * m2;   // float4 per system, both layouts
    const bool cv = S.A.complex_vals;
    hipEvent_t ev = prof_begin(st);
    for (int tr = 0; tr < 2; ++tr) {
        const int s0 = tr ? f.nright : 0, ns = tr ? nsys - f.nright : f.nright;
        if (ns <= 0) continue;
        dim3 grid(S.btiles_n, ns);
        const int2* tiles = (const int2*)S.btiles.p;
        const int* bc = (const int*)(tr ? S.bcolAT : S.bcolA).p;
        const void* bv = (tr ? S.bvalAT : S.bvalA).p;
        const float4* z = (const float4*)P + s0 * sysf4;
        float4* w = (float4*)f.W + s0 * sysf4;
        if (cv) {
            if (tr) k_spmm_blk<cf, true><<<grid, 256, sh, st>>>(n, m2, lpr, tiles, order, bc, (const cf*)bv,
                                                                f.shifts + s0, f.alpha, z, w);
            else k_spmm_blk<cf, false><<<grid, 256, sh, st>>>(n, m2, lpr, tiles, order, bc, (const cf*)bv,
                                                              f.shifts + s0, f.alpha, z, w);
        } else {
            k_spmm_blk<float, false><<<grid, 256, sh, st>>>(n, m2, lpr, tiles, order, bc, (const float*)bv,
                                                            f.shifts + s0, f.alpha, z, w);
        }
        FH_LAUNCH_CHECK();
    }
    if (ev) {
        const double vec = (double)nsys * n * m * sizeof(cf);
        const double ell = (double)n * SPMM_BLK_SL * (4.0 + (cv ? sizeof(cf) : sizeof(float))) + 4.0 * n;
        prof_end(st, ev, "spmm_blk_c64", 2 * vec + (f.nright < nsys && f.nright > 0 ? 2 : 1) * ell,
                 (double)nsys * m * 8.0 * (SPMM_BLK_SL + 1) * n);
    }
    return true;
}

template <typename T>
bool ilu_apply(hipStream_t st, const IluApplyArgs<T>& a, int nsys, Cx<T>* X, Cx<T>* Out, const T* scale,
               const SpmmAfter* after) {
    if (nsys <= 0) return false;
    FH_REQUIRE(scale == nullptr, -1, "ilu_apply: input scaling is not supported");
    dim3 grid(ceil_div(a.m, a.cw), nsys);
    const int K = std::max(std::max(a.fwd[0].K, a.bwd[0].K), std::max(a.fwd[1].K, a.bwd[1].K));
    // timing of the sweeps: X read, Out written by the forward sweep, read and
    // rewritten by the backward sweep; packed factor values and indices once
    // per system
    auto prof_sweep = [&](hipEvent_t e) {
        if (!e) return;
        const double vec = (double)nsys * a.n * a.m * sizeof(Cx<T>);
        const double fac = (double)a.n * (a.fwd[0].K + a.bwd[0].K) * (sizeof(Cx<T>) + 4) +
                           (double)a.n * (sizeof(Cx<T>) + 8);
        prof_end(st, e, std::string("ilu_apply_") + (sizeof(T) == 8 ? "c128" : "c64"), 4 * vec + nsys * fac,
                 (double)nsys * a.m * 8.0 * a.n * (a.fwd[0].K + a.bwd[0].K + 1));
    };
    hipEvent_t ev = prof_begin(st);
    bool lds = K <= 4;
    int wmax = 0, kmin = K;
    for (int sd = 0; sd < 2; ++sd) {
        lds = lds && a.fwd[sd].adjacent && a.bwd[sd].adjacent;
        wmax = std::max(wmax, std::max(a.fwd[sd].wmax, a.bwd[sd].wmax));
        kmin = std::min(kmin, std::min(a.fwd[sd].K, a.bwd[sd].K));
    }
    const size_t ring_bytes = 2 * sizeof(Cx<T>) * (size_t)wmax * a.cw;
    const size_t fac_bytes = 2 * (size_t)wmax * (2 * sizeof(Cx<T>) + sizeof(Cx<T>) + 2 * sizeof(int));
    // complex FP32, at most two off-diagonal slots, levels of at most 1,024
    // rows and 2,048 items, LDS within the device's per-workgroup limit: the
    // pipelined sweep (levels above 512 rows: two rows of factor data per
    // thread, and more than the default 64 KB of LDS)
    static int lds_max = -1;
    if (lds_max < 0) {
        int dev = 0, v = 0;
        FH_HIP(hipGetDevice(&dev));
        FH_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        lds_max = v;
    }
    const size_t sh = ring_bytes + fac_bytes;
    const bool pipe = lds && sizeof(T) == 4 && K <= 2 && kmin >= 1 && wmax <= 1024 && (long)wmax * a.cw <= 2048 &&
                      (long)a.n * a.m < (1L << 31) && a.n < (1 << 24) && a.m < (1 << 24) &&
                      sh <= (size_t)lds_max && a.junk != nullptr;
    // two columns per lane (16-byte accesses, factor data in registers) when
    // the column block is even, divides the row length (no partial block) and
    // a level's items fit one 512-thread batch of two items per thread
    static int vec_on = -1;
    if (vec_on < 0) {
        const char* e = std::getenv("FH_ILU_VEC");
        vec_on = e ? (std::atoi(e) != 0) : 1;
    }
    // (32-bit byte offsets: one system's block below 4 GB)
    const bool vec = pipe && vec_on && (a.cw == 2 || a.cw == 4 || a.cw == 8) && a.m % a.cw == 0 &&
                     (long)wmax * (a.cw / 2) <= 1024 && (long)a.n * a.m * 8 < (1L << 32);
    // blocked layout when a workgroup owns at most four columns of a row (a
    // row access of 32 bytes or less would be one short request per row):
    // permute in, sweep in place, permute back (tile of BLK_T rows in LDS)
    static int blk_on = -1;
    if (blk_on < 0) {
        const char* e = std::getenv("FH_ILU_BLK");
        blk_on = e ? (std::atoi(e) != 0) : 1;
    }
    const bool blocked = vec && blk_on && a.blk != nullptr && a.cw <= 4 &&
                         sizeof(float4) * BLK_T * (size_t)(a.m / 2 + 1) <= 65536;
    if (vec) {
        if constexpr (sizeof(T) == 4) {
            const int stride = wmax * (a.cw / 2);
            const size_t shv = 2 * sizeof(float4) * (size_t)stride;
            if (blocked) {
                // three launches, timed one by one: permutation in (the block
                // read and written once, plus the row order), the two sweeps
                // (the apply's own bytes, below), permutation out
                Cx<T>* P = (Cx<T>*)a.blk->ensure(sizeof(Cx<T>) * (size_t)nsys * a.n * a.m);
                const int* order = a.fwd[0].rows;    // the forward L sweep's packed order
                const double pbytes = 2.0 * nsys * a.n * a.m * sizeof(Cx<T>) + 4.0 * a.n;
                blk_perm(st, true, nsys, a.n, a.m, a.cw, order, X, P);   // timed from the event above
                prof_end(st, ev, "blk_perm_in_c64", pbytes);
                ev = prof_begin(st);
                if (a.cw == 2) k_ilu_apply_vec<2, 2, 512, 1, true><<<grid, 512, shv, st>>>(a, P, P, stride);
                else k_ilu_apply_vec<2, 2, 512, 2, true><<<grid, 512, shv, st>>>(a, P, P, stride);
                FH_LAUNCH_CHECK();
                prof_sweep(ev);
                // the operator product straight from the blocked layout
                if (after && spmm_after_blocked(st, *after, nsys, a.n, a.m, a.cw, order, P)) return true;
                ev = prof_begin(st);
                blk_perm(st, false, nsys, a.n, a.m, a.cw, order, P, Out);
                prof_end(st, ev, "blk_perm_out_c64", pbytes);
                return false;
            } else if (a.cw == 2) k_ilu_apply_vec<2, 2, 512, 1, false><<<grid, 512, shv, st>>>(a, X, Out, stride);
            else if (a.cw == 4) k_ilu_apply_vec<2, 2, 512, 2, false><<<grid, 512, shv, st>>>(a, X, Out, stride);
            else k_ilu_apply_vec<2, 2, 512, 4, false><<<grid, 512, shv, st>>>(a, X, Out, stride);
        }
    } else if (pipe) {
        if constexpr (sizeof(T) == 4) {
            const int stride = wmax * a.cw;
            auto go = [&](auto kern, int nt) {
                if (sh > 64 * 1024)
                    FH_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh));
                kern<<<grid, nt, sh, st>>>(a, X, Out, stride, wmax);
            };
            if (wmax > 512) go(k_ilu_apply_pipe<T, 4, 2, 512, 2>, 512);
            else if (wmax > 256 || (long)wmax * a.cw > 1024) go(k_ilu_apply_pipe<T, 4, 2, 512, 1>, 512);
            else go(k_ilu_apply_pipe<T, 4, 2, 256, 1>, 256);
        }
    } else if (lds && ring_bytes <= 48 * 1024) {
        // one batch per level when possible (a second batch would not be prefetched):
        // 512 threads when a level holds more than 256 x 4 items
        const int stride = wmax * a.cw;
        const bool wide = (long)wmax * a.cw > 256 * 4;
        const size_t sh = ring_bytes;
        if (K <= 2) {
            if (wide) k_ilu_apply_lds<T, 4, 2, 512><<<grid, 512, sh, st>>>(a, X, Out, stride);
            else k_ilu_apply_lds<T, 4, 2, 256><<<grid, 256, sh, st>>>(a, X, Out, stride);
        } else {
            if (wide) k_ilu_apply_lds<T, 4, 4, 512><<<grid, 512, sh, st>>>(a, X, Out, stride);
            else k_ilu_apply_lds<T, 4, 4, 256><<<grid, 256, sh, st>>>(a, X, Out, stride);
        }
    } else if (K <= 2) k_ilu_apply<T, 4, 2><<<grid, 256, 0, st>>>(a, X, Out);
    else if (K <= 4) k_ilu_apply<T, 4, 4><<<grid, 256, 0, st>>>(a, X, Out);
    else if (K <= 8) k_ilu_apply<T, 2, 8><<<grid, 256, 0, st>>>(a, X, Out);
    else if (K <= 32) k_ilu_apply<T, 1, 32><<<grid, 256, 0, st>>>(a, X, Out);
    else throw Error(-1, "ILU(0) sweeps support at most 32 off-diagonal entries per triangular row");
    FH_LAUNCH_CHECK();
    prof_sweep(ev);
    return false;
}
template bool ilu_apply<double>(hipStream_t, const IluApplyArgs<double>&, int, zd*, zd*, const double*,
                                const SpmmAfter*);
template bool ilu_apply<float>(hipStream_t, const IluApplyArgs<float>&, int, cf*, cf*, const float*,
                               const SpmmAfter*);

// Jacobi: Out = D^{-1} X (side 0) or D^{-H} X (side 1), D = diag(z - A) per node
template <typename T>
__global__ void k_jacobi(int n, int m, const int* __restrict__ node_of, const int* __restrict__ side_of,
                         const Cx<T>* __restrict__ dinv, Cx<T>* __restrict__ X, Cx<T>* __restrict__ Out,
                         const T* __restrict__ scale) {
    const int s = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const int i = e / m, c = e % m;
    const long base = (long)s * n * m;
    Cx<T> x = X[base + e];
    if (scale) { x = scale[(long)s * m + c] * x; X[base + e] = x; }
    if (!dinv) { Out[base + e] = x; return; }
    Cx<T> d = dinv[(long)node_of[s] * n + i];
    if (side_of[s]) d = conj(d);
    Out[base + e] = d * x;
}
template <typename T>
void jacobi_apply(hipStream_t st, const IluApplyArgs<T>& a, int nsys, Cx<T>* X, Cx<T>* Out, const T* scale) {
    dim3 grid(ceil_div((size_t)a.n * a.m, 256), nsys);
    k_jacobi<T><<<grid, 256, 0, st>>>(a.n, a.m, a.node_of, a.side_of, a.dinv, X, Out, scale);
    FH_LAUNCH_CHECK();
}
template void jacobi_apply<double>(hipStream_t, const IluApplyArgs<double>&, int, zd*, zd*, const double*);
template void jacobi_apply<float>(hipStream_t, const IluApplyArgs<float>&, int, cf*, cf*, const float*);

// ---------------------------------------------------------------------------
// GMRES building blocks (per column, all columns of all systems in lockstep)
// C = nsys * m columns; V_i at V + i * vstride (vstride = nsys*n*m)
// partial sums: part[(chunk * KMAXP + i) * C + col]
// ---------------------------------------------------------------------------
constexpr int ROWS_PER_CHUNK = 256;

// Load of a Krylov basis entry V_i (i < k) in the orthogonalization passes:
// each entry is read once per pass, so complex-FP32 loads are marked
// non-temporal (5.9 -> 5.7 ms per k <= 32 update pass, 4.8 -> 4.5 ms per dots
// pass).  The vectors just written by the previous kernel (V_k, W) keep
// ordinary loads: partly still in the last-level cache, they read slower
// non-temporally.
template <typename T>
__device__ __forceinline__ Cx<T> ld_basis(const Cx<T>* p) {
    if constexpr (sizeof(T) == 4) {
        const unsigned long long u = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
        Cx<T> r;
        __builtin_memcpy(&r, &u, sizeof(u));
        return r;
    } else {
        return *p;
    }
}

template <typename T> struct AccT { using type = double; };
template <> struct AccT<float> { using type = float; };

// per-chunk partial sums reduced over the ry row groups of the block through LDS
template <typename A, int KM>
__device__ __forceinline__ void store_partials(const A* acc_re, const A* acc_im, int kp1, int m, int c, int ty, int ry,
                                               int chunk, int C, int col, double* part, double (*sh)[256]) {
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        if (i < kp1) {
            sh[0][ty * m + c] = (double)acc_re[i];
            sh[1][ty * m + c] = (double)acc_im[i];
            __syncthreads();
            if (ty == 0) {
                double a = sh[0][c], b = sh[1][c];
                for (int t = 1; t < ry; ++t) { a += sh[0][t * m + c]; b += sh[1][t * m + c]; }
                part[((long)chunk * KM + i) * 2 * C + col] = a;
                part[((long)chunk * KM + i) * 2 * C + C + col] = b;
            }
            __syncthreads();
        }
    }
}

// h_i = V_i^H W  (i = 0..kp1-1); two rows per iteration (more loads in flight:
// 5.6 TB/s instead of 4.1 at 2,048 columns x 65,536 rows in complex FP32)
template <typename T, int KM>
__global__ __launch_bounds__(256) void k_cgs_dots(int n, int m, int kp1, const Cx<T>* __restrict__ V, long vstride,
                                                  const Cx<T>* __restrict__ W, double* __restrict__ part, int nchunk) {
    using A = typename AccT<T>::type;
    const int s = blockIdx.y, chunk = blockIdx.x;
    const int c = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const long base = (long)s * n * m;
    const int r0 = chunk * ROWS_PER_CHUNK, r1 = min(n, r0 + ROWS_PER_CHUNK);
    A acc_re[KM], acc_im[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) { acc_re[i] = A(0); acc_im[i] = A(0); }
    for (int r = r0 + ty; r < r1; r += 2 * ry) {
        const long off = base + (long)r * m + c;
        const bool two = r + ry < r1;
        const long off2 = two ? off + (long)ry * m : off;
        const Cx<T> w = W[off];
        const Cx<T> w2 = two ? W[off2] : czero<T>();
#pragma unroll
        for (int i = 0; i < KM; ++i) {
            if (i < kp1) {
                const Cx<T> v = V[i * vstride + off];
                const Cx<T> v2 = V[i * vstride + off2];
                acc_re[i] += (A)v.re * (A)w.re + (A)v.im * (A)w.im;
                acc_im[i] += (A)v.re * (A)w.im - (A)v.im * (A)w.re;
                acc_re[i] += (A)v2.re * (A)w2.re + (A)v2.im * (A)w2.im;
                acc_im[i] += (A)v2.re * (A)w2.im - (A)v2.im * (A)w2.re;
            }
        }
    }
    __shared__ double sh[2][256];
    store_partials<A, KM>(acc_re, acc_im, kp1, m, c, ty, ry, chunk, gridDim.y * m, s * m + c, part, sh);
}

// W' = W - sum_i h_i V_i ; then partial dots V_i^H W' (fused second pass).
// The kp1 values V_i of a row stay in registers between the update and the
// dots when they fit (complex FP32 up to 32 vectors, FP64 up to 16): V is
// read from HBM once.  Otherwise V_i is re-read (2.8x slower at 32 vectors:
// the re-reads miss the caches).
template <typename T, int KM>
__global__ __launch_bounds__(256) void k_cgs_update_dots(int n, int m, int kp1, const Cx<T>* __restrict__ V,
                                                         long vstride, Cx<T>* __restrict__ W,
                                                         const zd* __restrict__ h, double* __restrict__ part) {
    using A = typename AccT<T>::type;
    constexpr bool REGS = (sizeof(T) == 4 && KM <= 32) || (sizeof(T) == 8 && KM <= 16);
    const int s = blockIdx.y, chunk = blockIdx.x;
    const int c = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const long base = (long)s * n * m;
    const int C = gridDim.y * m;
    const int col = s * m + c;
    const int r0 = chunk * ROWS_PER_CHUNK, r1 = min(n, r0 + ROWS_PER_CHUNK);
    extern __shared__ unsigned char dsm[];
    Cx<T>* hs = reinterpret_cast<Cx<T>*>(dsm);          // [kp1][m] ([KM][m], zero-padded, for REGS)
    if (ty == 0) {
        for (int i = 0; i < kp1; ++i) hs[i * m + c] = ccast<T>(h[(long)i * C + col]);
        if constexpr (REGS)
            for (int i = kp1; i < KM; ++i) hs[i * m + c] = czero<T>();
    }
    __syncthreads();
    A acc_re[KM], acc_im[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) { acc_re[i] = A(0); acc_im[i] = A(0); }
    for (int r = r0 + ty; r < r1; r += ry) {
        const long off = base + (long)r * m + c;
        Cx<T> w = W[off];
        if constexpr (REGS) {
            // unconditional arithmetic (zero coefficients and values past kp1)
            // keeps the loads free of branches
            Cx<T> vv[KM];
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                vv[i] = (i < kp1) ? V[i * vstride + off] : czero<T>();
                cfms(w, hs[i * m + c], vv[i]);
            }
            W[off] = w;
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                acc_re[i] += (A)vv[i].re * (A)w.re + (A)vv[i].im * (A)w.im;
                acc_im[i] += (A)vv[i].re * (A)w.im - (A)vv[i].im * (A)w.re;
            }
        } else {
#pragma unroll
            for (int i = 0; i < KM; ++i)
                if (i < kp1) cfms(w, hs[i * m + c], V[i * vstride + off]);
            W[off] = w;
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                if (i < kp1) {
                    const Cx<T> v = V[i * vstride + off];
                    acc_re[i] += (A)v.re * (A)w.re + (A)v.im * (A)w.im;
                    acc_im[i] += (A)v.re * (A)w.im - (A)v.im * (A)w.re;
                }
            }
        }
    }
    __shared__ double sh[2][256];
    store_partials<A, KM>(acc_re, acc_im, kp1, m, c, ty, ry, chunk, C, col, part, sh);
}

// W'' = W' - sum_i h_i V_i ; partial ||W''||^2; two rows per iteration, the
// coefficients in registers when they fit
template <typename T, int KM>
__global__ __launch_bounds__(256) void k_cgs_update_norm(int n, int m, int kp1, const Cx<T>* __restrict__ V,
                                                         long vstride, Cx<T>* __restrict__ W,
                                                         const zd* __restrict__ h, double* __restrict__ part) {
    constexpr bool REGS = (sizeof(T) == 4 && KM <= 32) || (sizeof(T) == 8 && KM <= 16);
    const int s = blockIdx.y, chunk = blockIdx.x;
    const int c = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const long base = (long)s * n * m;
    const int C = gridDim.y * m;
    const int col = s * m + c;
    const int r0 = chunk * ROWS_PER_CHUNK, r1 = min(n, r0 + ROWS_PER_CHUNK);
    extern __shared__ unsigned char dsm[];
    Cx<T>* hs = reinterpret_cast<Cx<T>*>(dsm);          // [kp1][m]
    Cx<T> hr[REGS ? KM : 1];
    if constexpr (REGS) {
#pragma unroll
        for (int i = 0; i < KM; ++i) hr[i] = (i < kp1) ? ccast<T>(h[(long)i * C + col]) : czero<T>();
    } else {
        if (ty == 0)
            for (int i = 0; i < kp1; ++i) hs[i * m + c] = ccast<T>(h[(long)i * C + col]);
        __syncthreads();
    }
    double nn = 0.0;
    for (int r = r0 + ty; r < r1; r += 2 * ry) {
        const long off = base + (long)r * m + c;
        const bool two = r + ry < r1;
        const long off2 = two ? off + (long)ry * m : off;
        Cx<T> w = W[off];
        Cx<T> w2 = W[off2];
#pragma unroll
        for (int i = 0; i < KM; ++i)
            if (i < kp1) {
                const Cx<T> hi = REGS ? hr[REGS ? i : 0] : hs[i * m + c];
                cfms(w, hi, V[i * vstride + off]);
                cfms(w2, hi, V[i * vstride + off2]);
            }
        W[off] = w;
        nn += (double)w.re * w.re + (double)w.im * w.im;
        if (two) {
            W[off2] = w2;
            nn += (double)w2.re * w2.re + (double)w2.im * w2.im;
        }
    }
    __shared__ double sh[256];
    sh[ty * m + c] = nn;
    __syncthreads();
    if (ty == 0) {
        for (int t = 1; t < ry; ++t) nn += sh[t * m + c];
        part[(long)chunk * C + col] = nn;
    }
}

// column norms^2 of a block batch (partials)
template <typename T>
__global__ __launch_bounds__(256) void k_colnorm2(int n, int m, const Cx<T>* __restrict__ X, double* __restrict__ part) {
    const int s = blockIdx.y, chunk = blockIdx.x;
    const int c = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const long base = (long)s * n * m;
    const int C = gridDim.y * m;
    const int r0 = chunk * ROWS_PER_CHUNK, r1 = min(n, r0 + ROWS_PER_CHUNK);
    double nn = 0.0;
    for (int r = r0 + ty; r < r1; r += ry) {
        const Cx<T> w = X[base + (long)r * m + c];
        nn += (double)w.re * w.re + (double)w.im * w.im;
    }
    __shared__ double sh[256];
    sh[ty * m + c] = nn;
    __syncthreads();
    if (ty == 0) {
        for (int t = 1; t < ry; ++t) nn += sh[t * m + c];
        part[(long)chunk * C + s * m + c] = nn;
    }
}

// out[(i) * C + col] = sum_chunk part  (complex: two planes per i)
__global__ void k_reduce_dots(int nchunk, int kp1, int KM, int C, const double* __restrict__ part, zd* __restrict__ out,
                              int accumulate) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (col >= C || i >= kp1) return;
    double a = 0.0, b = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) {
        a += part[((long)ch * KM + i) * 2 * C + col];
        b += part[((long)ch * KM + i) * 2 * C + C + col];
    }
    zd v = cx(a, b);
    if (accumulate) v = v + out[(long)i * C + col];
    out[(long)i * C + col] = v;
}
__global__ void k_reduce_norm(int nchunk, int C, const double* __restrict__ part, double* __restrict__ out) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= C) return;
    double a = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) a += part[(long)ch * C + col];
    out[col] = sqrt(a);
}

template <typename T, int KM>
static void cgs_launch(hipStream_t st, int n, int m, int nsys, int kp1, const Cx<T>* V, long vstride, Cx<T>* W,
                       zd* h1, zd* h2, double* hnorm, DBuf& part, int passes) {
    const int ry = std::max(1, 256 / m);
    const int nchunk = ceil_div(n, ROWS_PER_CHUNK);
    const int C = nsys * m;
    double* P = (double*)part.ensure(sizeof(double) * (size_t)nchunk * KM * 2 * C);
    dim3 blk(m, ry), grid(nchunk, nsys);
    dim3 rg(ceil_div(C, 128), kp1);
    const double vec = (double)nsys * n * m * sizeof(Cx<T>);
    const std::string tag = std::string(sizeof(T) == 8 ? "c128" : "c64") + "_k" + std::to_string(KM);
    hipEvent_t ev = prof_begin(st);
    k_cgs_dots<T, KM><<<grid, blk, 0, st>>>(n, m, kp1, V, vstride, W, P, nchunk);
    FH_LAUNCH_CHECK();
    prof_end(st, ev, "cgs_dots_" + tag, (kp1 + 1) * vec, 8.0 * kp1 * vec / sizeof(Cx<T>));
    k_reduce_dots<<<rg, 128, 0, st>>>(nchunk, kp1, KM, C, P, h1, 0);
    FH_LAUNCH_CHECK();
    ev = prof_begin(st);
    const size_t hsb = sizeof(Cx<T>) * (size_t)kp1 * m;
    FH_REQUIRE(hsb <= 96 * 1024, -1, "GMRES restart length x columns per system too large for the LDS staging");
    constexpr bool REGS = (sizeof(T) == 4 && KM <= 32) || (sizeof(T) == 8 && KM <= 16);
    const size_t hsb_ud = REGS ? sizeof(Cx<T>) * (size_t)KM * m : hsb;   // zero-padded coefficients
    if (hsb > 64 * 1024) {
        FH_HIP(hipFuncSetAttribute((const void*)k_cgs_update_dots<T, KM>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
        FH_HIP(hipFuncSetAttribute((const void*)k_cgs_update_norm<T, KM>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024));
    }
    const zd* hlast = h1;
    if (passes >= 2) {
        k_cgs_update_dots<T, KM><<<grid, blk, hsb_ud, st>>>(n, m, kp1, V, vstride, W, h1, P);
        FH_LAUNCH_CHECK();
        prof_end(st, ev, "cgs_update_dots_" + tag, (kp1 + 2) * vec, 16.0 * kp1 * vec / sizeof(Cx<T>));
        k_reduce_dots<<<rg, 128, 0, st>>>(nchunk, kp1, KM, C, P, h2, 0);
        FH_LAUNCH_CHECK();
        ev = prof_begin(st);
        hlast = h2;
    } else {
        // one projection (classical Gram-Schmidt without the second pass): h2 = 0
        FH_HIP(hipMemsetAsync(h2, 0, sizeof(zd) * (size_t)kp1 * C, st));
    }
    k_cgs_update_norm<T, KM><<<grid, blk, hsb, st>>>(n, m, kp1, V, vstride, W, hlast, P);
    FH_LAUNCH_CHECK();
    prof_end(st, ev, "cgs_update_norm_" + tag, (kp1 + 2) * vec, 8.0 * kp1 * vec / sizeof(Cx<T>));
    k_reduce_norm<<<ceil_div(C, 128), 128, 0, st>>>(nchunk, C, P, hnorm);
    FH_LAUNCH_CHECK();
}

template <typename T>
void cgs2(hipStream_t st, int n, int m, int nsys, int kp1, const Cx<T>* V, long vstride, Cx<T>* W, zd* h1, zd* h2,
          double* hnorm, DBuf& part, int passes) {
    FH_REQUIRE(m >= 1 && m <= 256, -1, "GMRES column count per system must be in [1, 256]");
    if (kp1 <= 4) cgs_launch<T, 4>(st, n, m, nsys, kp1, V, vstride, W, h1, h2, hnorm, part, passes);
    else if (kp1 <= 8) cgs_launch<T, 8>(st, n, m, nsys, kp1, V, vstride, W, h1, h2, hnorm, part, passes);
    else if (kp1 <= 16) cgs_launch<T, 16>(st, n, m, nsys, kp1, V, vstride, W, h1, h2, hnorm, part, passes);
    else if (kp1 <= 32) cgs_launch<T, 32>(st, n, m, nsys, kp1, V, vstride, W, h1, h2, hnorm, part, passes);
    else if (kp1 <= 64) cgs_launch<T, 64>(st, n, m, nsys, kp1, V, vstride, W, h1, h2, hnorm, part, passes);
    else throw Error(-1, "GMRES restart length above 63 is not supported");
}
template void cgs2<double>(hipStream_t, int, int, int, int, const zd*, long, zd*, zd*, zd*, double*, DBuf&, int);
template void cgs2<float>(hipStream_t, int, int, int, int, const cf*, long, cf*, zd*, zd*, double*, DBuf&, int);

template <typename T>
void colnorms(hipStream_t st, int n, int m, int nsys, const Cx<T>* X, double* out, DBuf& part) {
    const int ry = std::max(1, 256 / m);
    const int nchunk = ceil_div(n, ROWS_PER_CHUNK);
    const int C = nsys * m;
    double* P = (double*)part.ensure(sizeof(double) * (size_t)nchunk * C);
    dim3 blk(m, ry), grid(nchunk, nsys);
    k_colnorm2<T><<<grid, blk, 0, st>>>(n, m, X, P);
    FH_LAUNCH_CHECK();
    k_reduce_norm<<<ceil_div(C, 128), 128, 0, st>>>(nchunk, C, P, out);
    FH_LAUNCH_CHECK();
}
template void colnorms<double>(hipStream_t, int, int, int, const zd*, double*, DBuf&);
template void colnorms<float>(hipStream_t, int, int, int, const cf*, double*, DBuf&);

// ---------------------------------------------------------------------------
// per-column Hessenberg column k: h = h1 + h2 (rows 0..k), h_{k+1} = ||w||;
// apply previous Givens rotations, form the new one, update g and the
// residual estimate |g_{k+1}|; 1/h_{k+1} is the scale of the next basis vector.
// State layout: Hs[(k * KP + i) * C + col] (column k of R), cs/sn[k * C + col],
// g[i * C + col].
// ---------------------------------------------------------------------------
// Givens update of Hessenberg column k of GMRES column `col`: Hs column k
// holds the new entries 0..k (not yet rotated), hn >= 0 is the subdiagonal
// entry h_{k+1,k}.  Applies the previous rotations, forms the new one, updates
// g and the residual estimate, and stops the column (kuse = k + 1) on
// convergence or breakdown.
__device__ void givens_col(int C, int k, int KP, int col, double hn, zd* __restrict__ Hs, double* __restrict__ cs,
                           zd* __restrict__ sn, zd* __restrict__ g, double* __restrict__ resid,
                           double* __restrict__ vscale, int* __restrict__ kuse, double bn, double tol) {
    zd* hc = Hs + (long)k * KP * C;
    // previous rotations
    for (int i = 0; i < k; ++i) {
        const double c = cs[(long)i * C + col];
        const zd s = sn[(long)i * C + col];
        const zd a = hc[(long)i * C + col], b = hc[(long)(i + 1) * C + col];
        zd na = c * a; cfma(na, s, b);
        zd nb = c * b; cfms(nb, conj(s), a);
        hc[(long)i * C + col] = na;
        hc[(long)(i + 1) * C + col] = nb;
    }
    // new rotation zeroing h_{k+1} = hn (real, >= 0)
    const zd x = hc[(long)k * C + col];
    const double ax = cabs(x);
    double c;
    zd s, r;
    if (hn == 0.0) { c = 1.0; s = czero<double>(); r = x; }
    else if (ax == 0.0) { c = 0.0; s = cx(1.0, 0.0); r = cx(hn, 0.0); }
    else {
        const double nrm = hypot(ax, hn);
        c = ax / nrm;
        const zd ph = cx(x.re / ax, x.im / ax);
        s = (hn / nrm) * ph;
        r = nrm * ph;
    }
    cs[(long)k * C + col] = c;
    sn[(long)k * C + col] = s;
    hc[(long)k * C + col] = r;
    const zd gk = g[(long)k * C + col];
    g[(long)k * C + col] = c * gk;
    const zd gk1 = -(conj(s) * gk);
    g[(long)(k + 1) * C + col] = gk1;
    const double res = cabs(gk1);
    resid[col] = res;
    // columns stop growing their basis after convergence or breakdown
    const bool stop = !(res > tol * bn && hn > 1e-300 * (ax + hn) && r.re == r.re);
    if (stop) kuse[col] = k + 1;
    vscale[col] = (hn > 0.0 && kuse[col] > k + 1) ? 1.0 / hn : 0.0;
}

__global__ void k_givens(int C, int k, int KP, const zd* __restrict__ h1, const zd* __restrict__ h2,
                         const double* __restrict__ hnorm, zd* __restrict__ Hs, double* __restrict__ cs,
                         zd* __restrict__ sn, zd* __restrict__ g, double* __restrict__ resid, double* __restrict__ vscale,
                         int* __restrict__ kuse, const double* __restrict__ bnorm, double tol) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= C) return;
    if (kuse[col] <= k) { vscale[col] = 0.0; return; }   // stopped earlier: keep its state
    zd* hc = Hs + (long)k * KP * C;
    for (int i = 0; i <= k; ++i) hc[(long)i * C + col] = h1[(long)i * C + col] + h2[(long)i * C + col];
    givens_col(C, k, KP, col, hnorm[col], Hs, cs, sn, g, resid, vscale, kuse, bnorm[col], tol);
}

// ---------------------------------------------------------------------------
// Delayed classical Gram-Schmidt with reorthogonalization (DCGS2) for the
// column-batched Arnoldi process: the second projection of the vector made at
// step k - 1 is deferred to step k, where its dot products share the pass
// over the basis with the first projection of the new vector.  Per step: one
// pass of dot products (reads V_0..V_k and W) and one update pass (reads them
// again, writes V_k and W), instead of three passes; the normalization is
// folded into the update.
//
// State entering step k >= 1 (per column): V_0..V_{k-1} orthonormal, V_k a
// tentative vector (once projected, scaled to about unit norm), the tentative
// Hessenberg column k - 1 (htent) and the scale tau with which the once
// projected vector t_k = tau V_k entered.  Dots of the pass:
//   s_i = V_i^H V_k, c_i = V_i^H W (i < k), alpha = V_k^H V_k, beta = V_k^H W,
//   omega = W^H W.
// With nu^2 = alpha - |s|^2 the reorthogonalized vector is
// (V_k - V s) / nu, the final column k - 1 is htent + tau s with subdiagonal
// tau nu, d = (c, (beta - s^H c) / nu) are the coefficients of W against the
// final V_0..V_k, and the new tentative vector is (W - V d) / rho with
// rho^2 = omega - |d|^2.  Its Hessenberg column: for the fixed (linear)
// preconditioner W was built from the tentative V_k, so the column is
// (d - H s) / nu with H the final columns 0..k-1 and tau = rho / nu; for the
// flexible variant W = A z_k belongs to z_k as it is, the column is d and
// tau = rho.
// ---------------------------------------------------------------------------
constexpr int DCGS_ROWS_PER_CHUNK = 1024;
// slots per chunk in the partial-dot buffer: s_0..s_{k-1}, c_0..c_{k-1},
// alpha, beta, omega for k <= 32
constexpr int DCGS_SLOTS = 2 * 32 + 3;

// A workgroup covers cb consecutive columns (of the m of a system; blockIdx.y
// = system * ncb + column block) and ry row groups; a thread owns one column.
// The launch handles basis vectors i0 .. i0 + KM - 1 (those below k), and
// alpha, beta, omega when extras != 0, so a pass over k vectors may be split
// into launches of KM vectors each (FP64: 16, to keep the accumulators in
// registers).
template <typename T, int KM>
__global__ __launch_bounds__(256) void k_dcgs_dots(int n, int m, int cb, int ncb, int k, int i0, int extras,
                                                   const Cx<T>* __restrict__ V, long vstride,
                                                   const Cx<T>* __restrict__ W, double* __restrict__ part) {
    using A = typename AccT<T>::type;
    constexpr int NE = 2 * KM + 3;
    const int s = blockIdx.y / ncb, cblk = blockIdx.y % ncb, chunk = blockIdx.x;
    const int tx = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const int c = cblk * cb + tx;
    const bool act = c < m;
    const long base = (long)s * n * m;
    const int C = (gridDim.y / ncb) * m;
    const int col = s * m + c;
    const int r0 = chunk * DCGS_ROWS_PER_CHUNK, r1 = act ? min(n, r0 + DCGS_ROWS_PER_CHUNK) : r0;
    const bool hw = W != nullptr;
    const int kl = min(KM, k - i0);             // basis vectors of this launch
    A sre[KM], sim[KM], cre[KM], cim[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) { sre[i] = A(0); sim[i] = A(0); cre[i] = A(0); cim[i] = A(0); }
    A al = A(0), bre = A(0), bim = A(0), om = A(0);
    const Cx<T>* Vk = V + (long)k * vstride;
    const Cx<T>* Vb = V + (long)i0 * vstride;
    for (int r = r0 + ty; r < r1; r += ry) {
        const long off = base + (long)r * m + c;
        const Cx<T> x = Vk[off];
        const Cx<T> w = hw ? W[off] : czero<T>();
        Cx<T> vv[KM];
#pragma unroll
        for (int i = 0; i < KM; ++i) vv[i] = (i < kl) ? ld_basis(Vb + i * vstride + off) : czero<T>();
#pragma unroll
        for (int i = 0; i < KM; ++i) {
            sre[i] += (A)vv[i].re * (A)x.re + (A)vv[i].im * (A)x.im;
            sim[i] += (A)vv[i].re * (A)x.im - (A)vv[i].im * (A)x.re;
            cre[i] += (A)vv[i].re * (A)w.re + (A)vv[i].im * (A)w.im;
            cim[i] += (A)vv[i].re * (A)w.im - (A)vv[i].im * (A)w.re;
        }
        if (extras) {
            al += (A)x.re * (A)x.re + (A)x.im * (A)x.im;
            bre += (A)x.re * (A)w.re + (A)x.im * (A)w.im;
            bim += (A)x.re * (A)w.im - (A)x.im * (A)w.re;
            om += (A)w.re * (A)w.re + (A)w.im * (A)w.im;
        }
    }
    // block reduction over the ry row groups, 8 entries per round; entry j of
    // the compact output order: s_0..s_{k-1}, c_0..c_{k-1}, alpha, beta, omega
    __shared__ double sh[8][2][256];
    const int t = ty * cb + tx;
#pragma unroll
    for (int g0 = 0; g0 < NE; g0 += 8) {
        // skip rounds whose entries are all unused (uniform over the block)
        bool any = false;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int slot = g0 + e;
            if (slot < NE) any = any || (slot < KM ? slot < kl : (slot < 2 * KM ? slot - KM < kl : extras != 0));
        }
        if (!any) continue;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int slot = g0 + e;
            double re = 0.0, im = 0.0;
            if (slot < KM) { re = sre[slot < KM ? slot : 0]; im = sim[slot < KM ? slot : 0]; }
            else if (slot < 2 * KM) { const int i = slot - KM; re = cre[i < KM && i >= 0 ? i : 0]; im = cim[i < KM && i >= 0 ? i : 0]; }
            else if (slot == 2 * KM) re = al;
            else if (slot == 2 * KM + 1) { re = bre; im = bim; }
            else if (slot == 2 * KM + 2) re = om;
            sh[e][0][t] = re;
            sh[e][1][t] = im;
        }
        __syncthreads();
        if (ty == 0 && act) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int slot = g0 + e;
                int j = -1;
                if (slot < KM) j = slot < kl ? i0 + slot : -1;
                else if (slot < 2 * KM) j = (slot - KM < kl) ? k + i0 + (slot - KM) : -1;
                else if (slot < NE) j = extras ? 2 * k + (slot - 2 * KM) : -1;
                if (j >= 0) {
                    double a = sh[e][0][tx], b = sh[e][1][tx];
                    for (int q = 1; q < ry; ++q) { a += sh[e][0][q * cb + tx]; b += sh[e][1][q * cb + tx]; }
                    part[((long)chunk * DCGS_SLOTS + j) * 2 * C + col] = a;
                    part[((long)chunk * DCGS_SLOTS + j) * 2 * C + C + col] = b;
                }
            }
        }
        __syncthreads();
    }
}

// Per-column scalars of DCGS2 step k (one thread per column).  D: reduced dots
// in the compact order.  Writes the update coefficients (coef rows [0, k): s,
// rows [KP, KP + k]: d), the scales scv = 1/nu (V_k) and scw = 1/rho (W), the
// final Hessenberg column k - 1 (Hraw unrotated; Hs then rotated by
// givens_col) and the tentative column k.  final != 0: only finalize column
// k - 1 (W absent).  Columns that have stopped get zero coefficients and
// scales, so their vectors become zero.
__global__ void k_dcgs_coef(int C, int k, int KP, int flex, int final, double floor_rel, const zd* __restrict__ D,
                            zd* __restrict__ Hraw, zd* __restrict__ Hs, double* __restrict__ cs, zd* __restrict__ sn,
                            zd* __restrict__ g, double* __restrict__ resid, double* __restrict__ vscale,
                            int* __restrict__ kuse, const double* __restrict__ bnorm, double tol,
                            zd* __restrict__ htent, double* __restrict__ tau, zd* __restrict__ coef,
                            double* __restrict__ scv, double* __restrict__ scw) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= C) return;
    auto dv = [&](int j) { return D[(long)j * C + col]; };
    auto zero_out = [&]() {
        for (int i = 0; i < k; ++i) coef[(long)i * C + col] = czero<double>();
        for (int i = 0; i <= k; ++i) coef[(long)(KP + i) * C + col] = czero<double>();
        scv[col] = 0.0;
        scw[col] = 0.0;
    };
    double nu = 1.0;
    if (k >= 1) {
        if (kuse[col] <= k - 1) { if (!final) zero_out(); return; }   // stopped earlier
        double s2 = 0.0;
        for (int i = 0; i < k; ++i) s2 += abs2(dv(i));
        const double alpha = dv(2 * k).re;
        const double nu2 = alpha - s2;
        nu = nu2 > floor_rel * alpha ? sqrt(nu2) : sqrt(floor_rel * alpha);
        if (!(nu > 0.0)) nu = 1.0;                                     // zero vector (breakdown)
        // final column k - 1: htent + tau s, subdiagonal tau nu
        const double tp = tau[col];
        zd* hr = Hraw + (long)(k - 1) * KP * C;
        zd* hc = Hs + (long)(k - 1) * KP * C;
        for (int i = 0; i < k; ++i) {
            zd v = htent[(long)i * C + col];
            cfma(v, cx(tp, 0.0), dv(i));
            hr[(long)i * C + col] = v;
            hc[(long)i * C + col] = v;
        }
        const double hn = tp * nu;
        hr[(long)k * C + col] = cx(hn, 0.0);
        givens_col(C, k - 1, KP, col, hn, Hs, cs, sn, g, resid, vscale, kuse, bnorm[col], tol);
        if (final) return;
        if (kuse[col] <= k) { zero_out(); return; }                    // converged at column k - 1
    } else if (kuse[col] <= 0) {
        zero_out();
        return;
    }
    // coefficients of W against the final V_0..V_k
    const int o = (k >= 1) ? k : 0;
    zd dk = (k >= 1) ? dv(2 * k + 1) : dv(1);
    for (int i = 0; i < k; ++i) {
        const zd ci = dv(o + i);
        dk = dk - conj(dv(i)) * ci;
        coef[(long)i * C + col] = dv(i);                 // s_i
        coef[(long)(KP + i) * C + col] = ci;             // d_i = c_i
    }
    dk = cx(dk.re / nu, dk.im / nu);
    coef[(long)(KP + k) * C + col] = dk;
    const double omega = (k >= 1) ? dv(2 * k + 2).re : dv(2).re;
    double d2 = abs2(dk);
    for (int i = 0; i < k; ++i) d2 += abs2(dv(o + i));
    const double rho2 = omega - d2;
    const double rho = rho2 > floor_rel * omega ? sqrt(rho2) : sqrt(floor_rel * omega);
    // tentative column k
    for (int l = 0; l <= k; ++l) {
        zd dl = (l < k) ? dv(o + l) : dk;
        if (!flex) {
            zd u = czero<double>();
            for (int i = (l > 0 ? l - 1 : 0); i < k; ++i) cfma(u, Hraw[((long)i * KP + l) * C + col], dv(i));
            dl = cx((dl.re - u.re) / nu, (dl.im - u.im) / nu);
        }
        htent[(long)l * C + col] = dl;
    }
    tau[col] = flex ? rho : rho / nu;
    scv[col] = 1.0 / nu;
    scw[col] = rho > 0.0 ? 1.0 / rho : 0.0;
}

// V_k <- (V_k - sum_{i<k} s_i V_i) scv ;  W <- (W - sum_{i<k} d_i V_i - d_k V_k) scw
// (workgroups over column blocks as in k_dcgs_dots)
template <typename T, int KM>
__global__ __launch_bounds__(256) void k_dcgs_update(int n, int m, int cb, int ncb, int k, Cx<T>* __restrict__ V,
                                                     long vstride, Cx<T>* __restrict__ W,
                                                     const zd* __restrict__ coef, int KP,
                                                     const double* __restrict__ scv, const double* __restrict__ scw) {
    const int s = blockIdx.y / ncb, cblk = blockIdx.y % ncb, chunk = blockIdx.x;
    const int tx = threadIdx.x, ty = threadIdx.y, ry = blockDim.y;
    const int c = cblk * cb + tx;
    const bool act = c < m;
    const long base = (long)s * n * m;
    const int C = (gridDim.y / ncb) * m;
    const int col = s * m + c;
    const int r0 = chunk * ROWS_PER_CHUNK, r1 = act ? min(n, r0 + ROWS_PER_CHUNK) : r0;
    extern __shared__ unsigned char dsm[];
    Cx<T>* hs = reinterpret_cast<Cx<T>*>(dsm);          // [KM][cb] s (zero-padded)
    Cx<T>* hd = hs + KM * cb;                           // [KM][cb] d (zero-padded)
    if (ty == 0) {
        for (int i = 0; i < KM; ++i) {
            hs[i * cb + tx] = (act && i < k) ? ccast<T>(coef[(long)i * C + col]) : czero<T>();
            hd[i * cb + tx] = (act && i < k) ? ccast<T>(coef[(long)(KP + i) * C + col]) : czero<T>();
        }
    }
    __syncthreads();
    if (!act) return;
    const Cx<T> dk = ccast<T>(coef[(long)(KP + k) * C + col]);
    const T sv = (T)scv[col], sw = (T)scw[col];
    Cx<T>* Vk = V + (long)k * vstride;
    for (int r = r0 + ty; r < r1; r += ry) {
        const long off = base + (long)r * m + c;
        Cx<T> x = Vk[off];
        Cx<T> w = W[off];
        // basis values in groups (FP64: 16 at a time, to stay within the
        // register file; FP32: all at once)
        constexpr int G = (sizeof(T) == 8 && KM > 16) ? 16 : KM;
#pragma unroll 1
        for (int g0 = 0; g0 < KM; g0 += G) {
            Cx<T> vv[G];
#pragma unroll
            for (int i = 0; i < G; ++i) vv[i] = (g0 + i < k) ? ld_basis(V + (g0 + i) * vstride + off) : czero<T>();
#pragma unroll
            for (int i = 0; i < G; ++i) {
                cfms(x, hs[(g0 + i) * cb + tx], vv[i]);
                cfms(w, hd[(g0 + i) * cb + tx], vv[i]);
            }
        }
        x.re *= sv;
        x.im *= sv;
        cfms(w, dk, x);
        w.re *= sw;
        w.im *= sw;
        if (k > 0) Vk[off] = x;
        W[off] = w;
    }
}

// column block of the DCGS2 kernels: all m columns when m <= 64, else 64 or 32
// columns (the last block of a system may be partial)
static int dcgs_colblock(int m) {
    if (m <= 64) return m;
    return (m % 64 == 0) ? 64 : ((m % 32 == 0) ? 32 : 64);
}

template <typename T, int KM>
static void dcgs_launch(hipStream_t st, int n, int m, int nsys, int k, Cx<T>* V, long vstride, Cx<T>* W,
                        const DcgsState& d, int flex, int final, double tol) {
    const int cb = dcgs_colblock(m), ncb = ceil_div(m, cb);
    const int ry = std::max(1, 256 / cb);
    const int C = nsys * m;
    const int nchunk_d = ceil_div(n, DCGS_ROWS_PER_CHUNK);
    double* P = (double*)d.part->ensure(sizeof(double) * (size_t)nchunk_d * DCGS_SLOTS * 2 * C);
    dim3 blk(cb, ry);
    const double vec = (double)nsys * n * m * sizeof(Cx<T>);
    const std::string tag = std::string(sizeof(T) == 8 ? "c128" : "c64") + "_k" + std::to_string(KM);
    const int ne = 2 * k + 3;
    // dots: FP64 accumulators for more than 16 vectors do not fit in
    // registers, so the pass is split into launches of 16 vectors (the block
    // vectors V_k and W are read once per launch)
    constexpr int KD = (sizeof(T) == 8 && KM > 16) ? 16 : KM;
    const int nl = std::max(1, (int)ceil_div(k, KD));
    for (int l = 0; l < nl; ++l) {
        const int i0 = l * KD, kl = std::max(0, std::min(KD, k - i0));
        hipEvent_t ev = prof_begin(st);
        k_dcgs_dots<T, KD><<<dim3(nchunk_d, nsys * ncb), blk, 0, st>>>(n, m, cb, ncb, k, i0, l == 0 ? 1 : 0, V,
                                                                        vstride, W, P);
        FH_LAUNCH_CHECK();
        prof_end(st, ev, "dcgs_dots_" + tag, (kl + (W ? 2 : 1)) * vec, 8.0 * (2 * kl + (l == 0 ? 3 : 0)) * vec / sizeof(Cx<T>));
    }
    k_reduce_dots<<<dim3(ceil_div(C, 128), ne), 128, 0, st>>>(nchunk_d, ne, DCGS_SLOTS, C, P, d.D, 0);
    FH_LAUNCH_CHECK();
    const double floor_rel = sizeof(T) == 4 ? 1e-7 : 1e-15;
    k_dcgs_coef<<<ceil_div(C, 128), 128, 0, st>>>(C, k, d.KP, flex, final, floor_rel, d.D, d.Hraw, d.Hs, d.cs, d.sn,
                                                   d.g, d.resid, d.vscale, d.kuse, d.bnorm, tol, d.htent, d.tau, d.coef,
                                                   d.scv, d.scw);
    FH_LAUNCH_CHECK();
    if (final) return;
    const int nchunk = ceil_div(n, ROWS_PER_CHUNK);
    const size_t lds = 2 * sizeof(Cx<T>) * (size_t)KM * cb;
    FH_REQUIRE(lds <= 64 * 1024, -1, "DCGS2: restart length x column block too large for the LDS staging");
    hipEvent_t ev = prof_begin(st);
    k_dcgs_update<T, KM><<<dim3(nchunk, nsys * ncb), blk, lds, st>>>(n, m, cb, ncb, k, V, vstride, W, d.coef, d.KP,
                                                                       d.scv, d.scw);
    FH_LAUNCH_CHECK();
    prof_end(st, ev, "dcgs_update_" + tag, (k + 2 + (k > 0 ? 2 : 1)) * vec, 16.0 * (k + 1) * vec / sizeof(Cx<T>));
}

template <typename T>
void dcgs_step(hipStream_t st, int n, int m, int nsys, int k, Cx<T>* V, long vstride, Cx<T>* W, const DcgsState& d,
               int flex, int final, double tol) {
    FH_REQUIRE(m >= 1 && m <= 256, -1, "GMRES column count per system must be in [1, 256]");
    if (k <= 4) dcgs_launch<T, 4>(st, n, m, nsys, k, V, vstride, W, d, flex, final, tol);
    else if (k <= 8) dcgs_launch<T, 8>(st, n, m, nsys, k, V, vstride, W, d, flex, final, tol);
    else if (k <= 16) dcgs_launch<T, 16>(st, n, m, nsys, k, V, vstride, W, d, flex, final, tol);
    else if (k <= 32) dcgs_launch<T, 32>(st, n, m, nsys, k, V, vstride, W, d, flex, final, tol);
    else throw Error(-1, "DCGS2: restart length above 32 is not supported");
}
template void dcgs_step<float>(hipStream_t, int, int, int, int, cf*, long, cf*, const DcgsState&, int, int, double);
template void dcgs_step<double>(hipStream_t, int, int, int, int, zd*, long, zd*, const DcgsState&, int, int, double);

// y = R^{-1} g (first kuse[col] steps), per column
__global__ void k_gmres_trisolve(int C, int k, int KP, const zd* __restrict__ Hs, const zd* __restrict__ g,
                                 const int* __restrict__ kuse, zd* __restrict__ y) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= C) return;
    const int ku = min(kuse[col], k);
    for (int i = ku; i < k; ++i) y[(long)i * C + col] = czero<double>();
    for (int i = ku - 1; i >= 0; --i) {
        zd s = g[(long)i * C + col];
        for (int j = i + 1; j < ku; ++j) cfms(s, Hs[((long)j * KP + i) * C + col], y[(long)j * C + col]);
        const zd d = Hs[((long)i * KP + i) * C + col];
        y[(long)i * C + col] = (d.re == 0.0 && d.im == 0.0) ? czero<double>() : cdiv(s, d);
    }
}

// U = sum_{i<k} y_i V_i   (per column)
template <typename T>
__global__ void k_combine(int n, int m, int k, const Cx<T>* __restrict__ V, long vstride, const zd* __restrict__ y,
                          Cx<T>* __restrict__ U) {
    const int s = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const int c = e % m;
    const int C = gridDim.y * m;
    const long off = (long)s * n * m + e;
    Cx<T> acc = czero<T>();
    for (int i = 0; i < k; ++i) cfma(acc, ccast<T>(y[(long)i * C + s * m + c]), V[i * vstride + off]);
    U[off] = acc;
}
template <typename T>
void gmres_update_prep(hipStream_t st, int n, int m, int nsys, int k, int KP, const zd* Hs, const zd* g,
                       const int* kuse, zd* y, const Cx<T>* V, long vstride, Cx<T>* U) {
    const int C = nsys * m;
    k_gmres_trisolve<<<ceil_div(C, 128), 128, 0, st>>>(C, k, KP, Hs, g, kuse, y);
    FH_LAUNCH_CHECK();
    dim3 grid(ceil_div((size_t)n * m, 256), nsys);
    k_combine<T><<<grid, 256, 0, st>>>(n, m, k, V, vstride, y, U);
    FH_LAUNCH_CHECK();
}
template void gmres_update_prep<double>(hipStream_t, int, int, int, int, int, const zd*, const zd*, const int*, zd*,
                                        const zd*, long, zd*);
template void gmres_update_prep<float>(hipStream_t, int, int, int, int, int, const zd*, const zd*, const int*, zd*,
                                       const cf*, long, cf*);

void givens_step(hipStream_t st, int C, int k, int KP, const zd* h1, const zd* h2, const double* hnorm, zd* Hs,
                 double* cs, zd* sn, zd* g, double* resid, double* vscale, int* kuse, const double* bnorm, double tol) {
    k_givens<<<ceil_div(C, 128), 128, 0, st>>>(C, k, KP, h1, h2, hnorm, Hs, cs, sn, g, resid, vscale, kuse, bnorm, tol);
    FH_LAUNCH_CHECK();
}

// start of a cycle: g = (beta, 0, ...), vscale = 1/beta, kuse = restart (or 0 if beta == 0 / converged)
__global__ void k_gmres_start(int C, int KP, int restart, const double* __restrict__ beta, const double* __restrict__ bnorm,
                              double tol, zd* __restrict__ g, double* __restrict__ vscale, int* __restrict__ kuse) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= C) return;
    const double b = beta[col];
    for (int i = 0; i < KP; ++i) g[(long)i * C + col] = czero<double>();
    g[col] = cx(b, 0.0);
    const bool done = !(b > tol * bnorm[col]) || !(b > 0.0);
    vscale[col] = done ? 0.0 : 1.0 / b;
    kuse[col] = done ? 0 : restart;
}
void gmres_start(hipStream_t st, int C, int KP, int restart, const double* beta, const double* bnorm, double tol, zd* g,
                 double* vscale, int* kuse) {
    k_gmres_start<<<ceil_div(C, 128), 128, 0, st>>>(C, KP, restart, beta, bnorm, tol, g, vscale, kuse);
    FH_LAUNCH_CHECK();
}

// X += Z (mixed: X FP64, Z in T)
template <typename T>
__global__ void k_add_to(long len, const Cx<T>* __restrict__ Z, zd* __restrict__ X) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) X[e] = X[e] + ccast<double>(Z[e]);
}
template <typename T>
void add_to(hipStream_t st, long len, const Cx<T>* Z, zd* X) {
    if (len <= 0) return;
    k_add_to<T><<<ceil_div(len, 256), 256, 0, st>>>(len, Z, X);
    FH_LAUNCH_CHECK();
}
template void add_to<double>(hipStream_t, long, const zd*, zd*);
template void add_to<float>(hipStream_t, long, const cf*, zd*);

// Z = X (same precision) for X in T
template <typename T>
__global__ void k_scale_cols_cast(int n, int m, const zd* __restrict__ X, const double* __restrict__ sc,
                                  Cx<T>* __restrict__ Out) {
    const int s = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const int c = e % m;
    const long off = (long)s * n * m + e;
    Out[off] = ccast<T>(sc[s * m + c] * X[off]);
}
template <typename T>
void scale_cols_cast(hipStream_t st, int n, int m, int nsys, const zd* X, const double* sc, Cx<T>* Out) {
    dim3 grid(ceil_div((size_t)n * m, 256), nsys);
    k_scale_cols_cast<T><<<grid, 256, 0, st>>>(n, m, X, sc, Out);
    FH_LAUNCH_CHECK();
}
template void scale_cols_cast<double>(hipStream_t, int, int, int, const zd*, const double*, zd*);
template void scale_cols_cast<float>(hipStream_t, int, int, int, const zd*, const double*, cf*);

// X += sc_col * Z
template <typename T>
__global__ void k_axpy_cols(int n, int m, const Cx<T>* __restrict__ Z, const double* __restrict__ sc, zd* __restrict__ X) {
    const int s = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const int c = e % m;
    const long off = (long)s * n * m + e;
    X[off] = X[off] + sc[s * m + c] * ccast<double>(Z[off]);
}
template <typename T>
void axpy_cols(hipStream_t st, int n, int m, int nsys, const Cx<T>* Z, const double* sc, zd* X) {
    dim3 grid(ceil_div((size_t)n * m, 256), nsys);
    k_axpy_cols<T><<<grid, 256, 0, st>>>(n, m, Z, sc, X);
    FH_LAUNCH_CHECK();
}
template void axpy_cols<double>(hipStream_t, int, int, int, const zd*, const double*, zd*);
template void axpy_cols<float>(hipStream_t, int, int, int, const cf*, const double*, zd*);

// ---------------------------------------------------------------------------
// residual-form filter accumulation:
//   Q[r][i] = rho_i Y[r][i] + sum_j c_{j,i} E_j[r][i]     (c_{j,i} = w_j/(z_j - lam_i), conj for left)
// coef: [ne][m] complex; E: [ne][n][m] (system-major slice of one side)
// ---------------------------------------------------------------------------
__global__ void k_filter_accum(int ne, int n, int m, const zd* __restrict__ E, const zd* __restrict__ coef,
                               const zd* __restrict__ Y, const zd* __restrict__ rho, int add, zd* __restrict__ Q) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const int c = e % m;
    zd acc = add ? Q[e] : czero<double>();
    if (Y) cfma(acc, rho[c], Y[e]);
    for (int j = 0; j < ne; ++j) cfma(acc, coef[(long)j * m + c], E[(long)j * n * m + e]);
    Q[e] = acc;
}
void filter_accum(hipStream_t st, int ne, int n, int m, const zd* E, const zd* coef, const zd* Y, const zd* rho, zd* Q,
                  bool add) {
    k_filter_accum<<<ceil_div((size_t)n * m, 256), 256, 0, st>>>(ne, n, m, E, coef, Y, rho, add ? 1 : 0, Q);
    FH_LAUNCH_CHECK();
}

// Conjugation-closed columns: E_j (j < ne) are the solutions at the upper
// nodes only.  Column c of the lower partner of node j is conj(E_j[:, cp[c]]),
// so Q[:, c] += cu_j[c] E_j[:, c] + cl_j[c] conj(E_j[:, cp[c]]).
__global__ void k_filter_accum_pair(int ne, int n, int m, const zd* __restrict__ E, const zd* __restrict__ cu,
                                    const zd* __restrict__ cl, const int* __restrict__ cp, const zd* __restrict__ Y,
                                    const zd* __restrict__ rho, int add, zd* __restrict__ Q) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const int c = e % m;
    const long ep = e - c + cp[c];
    zd acc = add ? Q[e] : czero<double>();
    if (Y) cfma(acc, rho[c], Y[e]);
    for (int j = 0; j < ne; ++j) {
        const zd* Ej = E + (long)j * n * m;
        cfma(acc, cu[(long)j * m + c], Ej[e]);
        cfma(acc, cl[(long)j * m + c], conj(Ej[ep]));
    }
    Q[e] = acc;
}
void filter_accum_pair(hipStream_t st, int ne, int n, int m, const zd* E, const zd* cu, const zd* cl, const int* cp,
                       const zd* Y, const zd* rho, zd* Q, bool add) {
    k_filter_accum_pair<<<ceil_div((size_t)n * m, 256), 256, 0, st>>>(ne, n, m, E, cu, cl, cp, Y, rho, add ? 1 : 0,
                                                                        Q);
    FH_LAUNCH_CHECK();
}

// flag = 1 if any entry of X (len) has a nonzero imaginary part (flag zeroed by the caller)
__global__ void k_any_imag(long len, const zd* __restrict__ X, int* __restrict__ flag) {
    int any = 0;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (long)gridDim.x * blockDim.x)
        any |= X[e].im != 0.0;
    if (__any(any) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}
void any_imag(hipStream_t st, long len, const zd* X, int* flag_dev) {
    if (len <= 0) return;
    const int grid = (int)std::min<long>(ceil_div(len, 256), 4096);
    k_any_imag<<<grid, 256, 0, st>>>(len, X, flag_dev);
    FH_LAUNCH_CHECK();
}

// R = A Y - Y diag(lam)  (left: A^H Yh - Yh diag(conj lam)); computed as
// spmm with shifts per column -> use a column-shift variant
template <typename TA, bool CONJ>
__global__ void k_spmm_colshift(int n, int m, const int* __restrict__ rowptr, const int* __restrict__ col,
                                const TA* __restrict__ val, const zd* __restrict__ lam, int conj_lam,
                                const zd* __restrict__ X, zd* __restrict__ Out) {
    const int r = blockIdx.x * blockDim.y + threadIdx.y;
    const int c = threadIdx.x;
    if (r >= n) return;
    zd acc = czero<double>();
    const int p1 = rowptr[r + 1];
    for (int p = rowptr[r]; p < p1; ++p) mac_val(acc, val[p], X[(long)col[p] * m + c], CONJ);
    zd l = lam[c];
    if (conj_lam) l = conj(l);
    cfms(acc, l, X[(long)r * m + c]);
    Out[(long)r * m + c] = acc;
}
void ritz_residual(hipStream_t st, const CsrDev& A, bool conj_t, int n, int m, const zd* lam, bool conj_lam,
                   const zd* X, zd* Out) {
    const int ry = m >= 256 ? 1 : std::max(1, 256 / m);
    dim3 blk(m, ry), grid(ceil_div(n, ry));
    if (A.complex_vals) {
        if (conj_t) k_spmm_colshift<zd, true><<<grid, blk, 0, st>>>(n, m, A.rowptr, A.col, (const zd*)A.val64, lam, conj_lam, X, Out);
        else k_spmm_colshift<zd, false><<<grid, blk, 0, st>>>(n, m, A.rowptr, A.col, (const zd*)A.val64, lam, conj_lam, X, Out);
    } else {
        k_spmm_colshift<double, false><<<grid, blk, 0, st>>>(n, m, A.rowptr, A.col, (const double*)A.val64, lam, conj_lam, X, Out);
    }
    FH_LAUNCH_CHECK();
}

// dst[q] = src[idx[q]]  (FP64 real or complex values)
template <typename V>
__global__ void k_gather(long len, const V* __restrict__ src, const int* __restrict__ idx, V* __restrict__ dst) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) dst[e] = src[idx[e]];
}
void gather_vals(hipStream_t st, long len, bool complex_vals, const void* src, const int* idx, void* dst) {
    if (len <= 0) return;
    if (complex_vals) k_gather<zd><<<ceil_div(len, 256), 256, 0, st>>>(len, (const zd*)src, idx, (zd*)dst);
    else k_gather<double><<<ceil_div(len, 256), 256, 0, st>>>(len, (const double*)src, idx, (double*)dst);
    FH_LAUNCH_CHECK();
}
__global__ void k_cast_real(long len, const double* __restrict__ s, float* __restrict__ d) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) d[e] = (float)s[e];
}
void cast_vals(hipStream_t st, long len, bool complex_vals, const void* src, void* dst) {
    if (len <= 0) return;
    if (complex_vals) k_cast_d<float><<<ceil_div(len, 256), 256, 0, st>>>(len, (const zd*)src, (cf*)dst);
    else k_cast_real<<<ceil_div(len, 256), 256, 0, st>>>(len, (const double*)src, (float*)dst);
    FH_LAUNCH_CHECK();
}

// jd[j][i] = 1 / M_j[i][i] from the (unfactored) values on the M pattern
__global__ void k_jacobi_diag(int n, long nnzM, const int* __restrict__ diag, const zd* __restrict__ mv, zd* __restrict__ jd) {
    const int j = blockIdx.y;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) jd[(long)j * n + i] = cdiv(cx(1.0, 0.0), mv[(long)j * nnzM + diag[i]]);
}
void jacobi_diag(hipStream_t st, const SparseState& S, int ne, const zd* mvals, zd* jd) {
    dim3 g(ceil_div(S.n, 256), ne);
    k_jacobi_diag<<<g, 256, 0, st>>>(S.n, S.nnzM, S.mdiag, mvals, jd);
    FH_LAUNCH_CHECK();
}
__global__ void k_invert(long len, zd* __restrict__ v) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) v[e] = cdiv(cx(1.0, 0.0), v[e]);
}
void invert_vals(hipStream_t st, long len, zd* v) {
    if (len <= 0) return;
    k_invert<<<ceil_div(len, 256), 256, 0, st>>>(len, v);
    FH_LAUNCH_CHECK();
}
// X[s][r][c] *= sc[s*m + c]
template <typename T>
__global__ void k_scale_inplace(int n, int m, Cx<T>* __restrict__ X, const double* __restrict__ sc) {
    const int s = blockIdx.y;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * m) return;
    const long off = (long)s * n * m + e;
    X[off] = T(sc[s * m + (e % m)]) * X[off];
}
template <typename T>
void scale_inplace(hipStream_t st, int n, int m, int nsys, Cx<T>* X, const double* sc) {
    dim3 grid(ceil_div((size_t)n * m, 256), nsys);
    k_scale_inplace<T><<<grid, 256, 0, st>>>(n, m, X, sc);
    FH_LAUNCH_CHECK();
}
template void scale_inplace<double>(hipStream_t, int, int, int, zd*, const double*);
template void scale_inplace<float>(hipStream_t, int, int, int, cf*, const double*);
template <typename T>
__global__ void k_add_same(long len, const Cx<T>* __restrict__ Z, Cx<T>* __restrict__ X) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < len) X[e] = X[e] + Z[e];
}
template <typename T>
void add_same(hipStream_t st, long len, const Cx<T>* Z, Cx<T>* X) {
    if (len <= 0) return;
    k_add_same<T><<<ceil_div(len, 256), 256, 0, st>>>(len, Z, X);
    FH_LAUNCH_CHECK();
}
template void add_same<double>(hipStream_t, long, const zd*, zd*);
template void add_same<float>(hipStream_t, long, const cf*, cf*);

}  // namespace fh
