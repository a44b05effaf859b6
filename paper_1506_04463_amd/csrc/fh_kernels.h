// Host-side launchers of the feasthip HIP kernels (gfx950).
#pragma once
#include "fh_common.h"

namespace fh {

// ----------------------------- k_blas.hip ----------------------------------
// C = alpha op(A) op(B) + beta C, row-major, batched (blockIdx.z) with strides.
// opA/opB: 'N' or 'C' (conjugate transpose).
template <typename T>
void gemm(hipStream_t st, char opA, char opB, int M, int N, int K, Cx<T> alpha, const Cx<T>* A, long lda,
          long sA, const Cx<T>* B, long ldb, long sB, Cx<T> beta, Cx<T>* C, long ldc, long sC, int batch);

// C (p x q) = X^H Y for tall n x p X and n x q Y (row-major), split over n and
// reduced in a fixed order (deterministic).
void gemm_hn_tall(hipStream_t st, int n, int p, int q, const zd* X, long ldx, const zd* Y, long ldy, zd* C,
                  long ldc, DBuf& partial);
// The same product with the partial sums in caller-provided device memory of
// cap bytes (nothing allocated).  The split over n is the one gemm_hn_tall
// uses when its partials fit in cap, else a coarser one.  Returns false (and
// launches nothing) when not even one p x q partial fits.
bool gemm_hn_tall_into(hipStream_t st, int n, int p, int q, const zd* X, long ldx, const zd* Y, long ldy, zd* C,
                       long ldc, void* part, size_t cap);

// Column 1-norms for eq:res: num_c = sum_i |AY_ic - lam_c BY_ic|,
// den_c = sum_i |BY_ic| over an n x m block (ld).  lam: device, m.
void res_colnorms(hipStream_t st, int n, int m, const zd* AY, const zd* BY, long ld, const zd* lam,
                  bool conj_lam, double* num, double* den, DBuf& partial);

// Q = sum_j c_j X_j   with c_j = w_j (or conj(w_j) when conj_w), X_j at X + j*strideX
void accumulate(hipStream_t st, int ne, long len, const zd* X, long strideX, const zd* w_dev, bool conj_w,
                zd* Q);

// dst_j = src for j = 0..copies-1 (stride len)
template <typename T>
void replicate(hipStream_t st, long len, const Cx<T>* src, Cx<T>* dst, int copies);

// dst = conj(src), elementwise
void conj_copy(hipStream_t st, long len, const zd* src, zd* dst);
// Qh = conj(Q) diag(conj(1 / s)), s_c = sum_r Y[r][c]^2 (n x m row-major blocks):
// the filter of the left block conj(Y) D that satisfies yh_c^H y_c = 1
void conj_copy_bilin(hipStream_t st, int n, int m, const zd* Y, const zd* Q, zd* Qh, DBuf& part);

// Make the columns of X (n x m) closed under conjugation, in place: cp_dev is
// an involution on the columns; a pair (i, k = cp[i] > i) gets x_k = conj(x_i),
// a column with cp[c] = c is rotated by the phase that makes x_c^T x_c real
// positive and its imaginary part dropped.  Xh (or nullptr) takes the same
// operations with X's phases.
void conj_close_cols(hipStream_t st, int n, int m, zd* X, zd* Xh, const int* cp_dev, DBuf& part);
// X = Re(X) in place (len entries)
void real_part(hipStream_t st, long len, zd* X);

// cast between complex precisions
template <typename D, typename S>
void cast(hipStream_t st, long len, const Cx<S>* src, Cx<D>* dst);

// Out = s X - Out (elementwise, len entries)
void shift_combine(hipStream_t st, long len, zd s, const zd* X, zd* Out);

// Out = A - B (elementwise, len entries)
void sub(hipStream_t st, long len, const zd* A, const zd* B, zd* Out);

// dst[i][k] = src[i][perm[k]] for k < mout (rows n; lds, ldd leading dims)
void gather_cols(hipStream_t st, int n, int mout, const zd* src, long lds, const int* perm_dev, zd* dst,
                 long ldd);

// ----------------------------- k_dense.hip ---------------------------------
// M_j = z_j B - A (B == nullptr: identity) for j = 0..ne-1, stride n*n, ld n
void form_shift(hipStream_t st, int n, const zd* A, long lda, const zd* B, long ldb, int ne, const zd* z_dev,
                zd* M);
// LU with partial pivoting of `batch` n x n matrices (stride n*n, ld n), in place.
// ipiv: batch*n (0-based), info: batch (0 or first zero pivot + 1).
void lu_factor(hipStream_t st, int n, zd* M, int batch, int* ipiv, int* info, DBuf& scratch);
// Solve op(M_j) X_j = X_j (op 'N' or 'C'), X_j n x m (ld m), stride n*m.
void lu_solve(hipStream_t st, char op, int n, const zd* M, const int* ipiv, int m, zd* X, int batch);

// ----------------------------- k_eig.hip -----------------------------------
// one small eigenproblem of a batched launch (fields used by each kernel:
// biortho: m, in1 = B_Q, eta, out0 = gamma, out1 = S, out2 = Sh, i0 = m0t, i1 = info;
// reduced: m, in1 = A_U, in2 = B_U, out0 = lambda, out1 = W, out2 = Wh, i0 = info)
struct EigJob {
    int m;
    double eta;
    const zd* in1;
    const zd* in2;
    zd* out0;
    zd* out1;
    zd* out2;
    int* i0;
    int* i1;
    zd* work;      // eig_work_size(m) bytes
};
size_t eig_work_size(int m);
void eig_biortho_batched(hipStream_t st, int count, const EigJob* jobs_dev, int mmax);
void eig_reduced_batched(hipStream_t st, int count, const EigJob* jobs_dev, int mmax);
// Steps 3.a-3.c (see fh_biortho_factors); work: device scratch
void eig_biortho(hipStream_t st, int m, const zd* BQ, double eta, zd* gamma, zd* S, zd* Sh, int* m0t,
                 int* info, DBuf& work);
// Step 4.b (see fh_reduced_eig)
void eig_reduced(hipStream_t st, int m, const zd* AU, const zd* BU, zd* lam, zd* W, zd* Wh, int* info,
                 DBuf& work);

}  // namespace fh
