// Sparse (CSR) state of a prepared problem and launchers of k_sparse.hip.
#pragma once
#include <vector>

#include "fh_internal.h"

namespace fh {

// CSR operand on the device; values in FP64 (val64) and an FP32 copy (val32)
struct CsrDev {
    const int* rowptr = nullptr;
    const int* col = nullptr;
    const void* val64 = nullptr;
    const void* val32 = nullptr;
    bool complex_vals = false;
    long nnz = 0;
    int maxrow = 0;   // longest row (entries)
    template <typename T> const void* val() const { return sizeof(T) == sizeof(double) ? val64 : val32; }
};

struct LevelsDev {
    const int* ptr = nullptr;    // nlev + 1
    const int* rows = nullptr;   // n
    int nlev = 0;
};

// One triangular sweep in level-packed ELL form: packed row t (level order)
// is matrix row rows[t]; its off-diagonal entries sit in slots k < K at
// ell_col[k*n + t] (-1 = empty) with per-node values ell_val[node][k*n + t];
// a non-unit sweep multiplies by dval[node][t] (the inverse pivot).
struct SweepDev {
    const int* lev_ptr = nullptr;   // nlev + 1
    const int* rows = nullptr;      // n
    const int* ell_col = nullptr;   // K * n
    const int* ell_pos = nullptr;   // K * n: position of the value in the LU factor (-1 = empty)
    const int* dpos = nullptr;      // n: position of the pivot (non-unit sweeps) or null
    const int* ell_slot = nullptr;  // K * n: position of the dependency within the previous level (-1: none)
    const int* ppos = nullptr;      // n: position of the row in the forward L sweep's packed order (the order
                                    // of the blocked vector layout of the two-column sweep)
    int nlev = 0, K = 0;
    int wmax = 0;                   // widest level (rows)
    bool adjacent = false;          // every dependency lies in the level just before
    bool pad_ = false;
    bool conj = false;              // values enter conjugated (left-side sweeps)
};

template <typename T>
struct IluApplyArgs {
    int n = 0, m = 0, cw = 8;
    const int* node_of = nullptr;  // per system
    const int* side_of = nullptr;  // per system
    SweepDev fwd[2], bwd[2];       // [side]: side 0 = L then U, side 1 = U^H then L^H
    const Cx<T>* fval[2] = {nullptr, nullptr};   // [node][K*n]
    const Cx<T>* fdiag[2] = {nullptr, nullptr};  // [node][n] or null (unit)
    const Cx<T>* bval[2] = {nullptr, nullptr};
    const Cx<T>* bdiag[2] = {nullptr, nullptr};
    const Cx<T>* dinv = nullptr;                 // Jacobi: [node][n] (null: identity)
    Cx<T>* junk = nullptr;   // write target of the pipelined sweep's fill and drain levels
                             // (ILU_JUNK entries, written by every workgroup, never read)
    DBuf* blk = nullptr;     // workspace of the blocked layout (nsys x n x m entries, grown on use;
                             // null: natural layout only)
};
constexpr int ILU_JUNK = 4096;

struct NetState;

struct SparseState {
    int n = 0;
    long nnzA = 0, nnzM = 0;
    bool csym = false;            // A = A^T (pattern and values)
    CsrDev A, AT;
    // M = A + diagonal pattern and its transpose
    int *mrowptr = nullptr, *mcol = nullptr, *mdiag = nullptr, *a2m = nullptr;
    int *trowptr = nullptr, *tcol = nullptr, *tdiag = nullptr, *t2m = nullptr;
    int* uptr = nullptr;
    int2* upd = nullptr;
    long nupd = 0;
    LevelsDev levL, levU, levUT, levLT;
    SweepDev swL, swU, swUT, swLT;
    std::vector<DBuf*> owned;     // every device array above
    // factor cache
    std::vector<cplx> fact_z;
    int fact_prec = -1;
    DBuf lu64, luT64, dinv64, jd64, lu32, luT32, dinv32, jd32, mvals, zdev;
    DBuf pk64[6], pk32[6];          // packed sweep values: L, U, Udiag, UT, UTdiag, LT
    int ilu_cw64 = 4, ilu_cw32 = 8;  // columns per workgroup of the ILU sweeps (measured best at m = 64)
    // batch descriptors and GMRES workspace
    DBuf junk;   // see IluApplyArgs::junk
    DBuf blk;    // see IluApplyArgs::blk
    DBuf node_of, side_of, shifts64, shifts32, coef, rho, bufB, bufX, bufR, bufT, b32, x32;
    DBuf V, Z, Hs, cs, sn, g, resid, vscale, kuse, y, h1, h2, hnorm, beta, bnorm, part, bn64, rn64, sc64;
    DBuf Hraw, htent, tau, dcoef, scv, scw, dots;   // DCGS2
    DBuf cpd, coefp, flag;   // conjugation-closed filter: column partners, upper/lower weights, real-input flag
    DBuf aval32, atval64, atval32, bn32, Zf;
    // the operator's rows in the blocked layout's position order (ELL with
    // SPMM_BLK_SL slots: neighbour positions and FP32 values, of A and of
    // A^T), built on first use by the product that reads the blocked sweep's
    // output (ilu_apply with SpmmAfter)
    DBuf bpos, bcolA, bvalA, bcolAT, bvalAT;
    DBuf btiles;           // int2 (first position, count) per workgroup of that product
    int btiles_n = 0;
    bool bell_ready = false;
    NetState* net = nullptr;   // attached learned preconditioner (not owned)
    ~SparseState() {
        for (DBuf* b : owned) delete b;
    }
};

// k_sparse.hip launchers
template <typename T>
void spmm(hipStream_t st, const CsrDev& A, bool conj_t, int n, int m, int nsys, const Cx<T>* shifts, T alpha,
          const Cx<T>* X, const Cx<T>* Yadd, Cx<T>* Out);
void form_mvals(hipStream_t st, const SparseState& S, int ne, const zd* z_dev, zd* out);
void ilu0_factor(hipStream_t st, const SparseState& S, int ne, zd* lu, zd* luT, zd* dinv);
void pack_sweep_vals(hipStream_t st, const SweepDev& sw, int n, int ne, long nnzM, const zd* lu, zd* ell, zd* diag);
void to_single(hipStream_t st, long len, const zd* s, cf* d);
// The operator product that follows the preconditioner in a Krylov step,
// W_s = alpha (sh_s Z_s - op(A) Z_s) for Z = the preconditioner's output
// (systems [0, nright) with A, the rest with A^H, as apply_M).  Given to
// ilu_apply, it is computed straight from the blocked layout of the
// two-column sweep when that layout is used (no move of Z back to the
// natural layout); ilu_apply then returns true and Out is not written.
struct SpmmAfter {
    SparseState* S = nullptr;
    int nright = 0;
    const cf* shifts = nullptr;
    float alpha = 1.f;
    cf* W = nullptr;
};
constexpr int SPMM_BLK_SL = 5;
template <typename T>
bool ilu_apply(hipStream_t st, const IluApplyArgs<T>& a, int nsys, Cx<T>* X, Cx<T>* Out, const T* scale,
               const SpmmAfter* after = nullptr);
template <typename T>
void jacobi_apply(hipStream_t st, const IluApplyArgs<T>& a, int nsys, Cx<T>* X, Cx<T>* Out, const T* scale);
template <typename T>
void cgs2(hipStream_t st, int n, int m, int nsys, int kp1, const Cx<T>* V, long vstride, Cx<T>* W, zd* h1, zd* h2,
          double* hnorm, DBuf& part, int passes);
// Device state of the delayed-reorthogonalization Arnoldi step (DCGS2): the
// GMRES arrays it updates (Hs rotated, cs, sn, g, resid, vscale, kuse, bnorm)
// and its own (Hraw unrotated columns [restart][KP][C], htent [KP][C], tau,
// coef [2 KP][C], scv, scw, D reduced dots [2 KM + 3][C], part partials).
struct DcgsState {
    int KP = 0;
    zd *Hs = nullptr, *sn = nullptr, *g = nullptr, *Hraw = nullptr, *htent = nullptr, *coef = nullptr, *D = nullptr;
    double *cs = nullptr, *resid = nullptr, *vscale = nullptr, *tau = nullptr, *scv = nullptr, *scw = nullptr;
    const double* bnorm = nullptr;
    int* kuse = nullptr;
    DBuf* part = nullptr;
};
// Step k of DCGS2 Arnoldi (complex FP32 or FP64 basis, k <= 32): W = A z_k holds the
// new vector on entry; V_k is reorthogonalized in place and W becomes the
// tentative V_{k+1}; Hessenberg column k - 1 is finalized and rotated.
// final != 0 (W = nullptr): only finalize column k - 1.
template <typename T>
void dcgs_step(hipStream_t st, int n, int m, int nsys, int k, Cx<T>* V, long vstride, Cx<T>* W, const DcgsState& d,
               int flex, int final, double tol);
template <typename T>
void colnorms(hipStream_t st, int n, int m, int nsys, const Cx<T>* X, double* out, DBuf& part);
void givens_step(hipStream_t st, int C, int k, int KP, const zd* h1, const zd* h2, const double* hnorm, zd* Hs,
                 double* cs, zd* sn, zd* g, double* resid, double* vscale, int* kuse, const double* bnorm, double tol);
void gmres_start(hipStream_t st, int C, int KP, int restart, const double* beta, const double* bnorm, double tol, zd* g,
                 double* vscale, int* kuse);
template <typename T>
void gmres_update_prep(hipStream_t st, int n, int m, int nsys, int k, int KP, const zd* Hs, const zd* g,
                       const int* kuse, zd* y, const Cx<T>* V, long vstride, Cx<T>* U);
template <typename T>
void add_to(hipStream_t st, long len, const Cx<T>* Z, zd* X);
template <typename T>
void scale_cols_cast(hipStream_t st, int n, int m, int nsys, const zd* X, const double* sc, Cx<T>* Out);
template <typename T>
void axpy_cols(hipStream_t st, int n, int m, int nsys, const Cx<T>* Z, const double* sc, zd* X);
// Q = (add ? Q : 0) + Y diag(rho) (when Y) + sum_j E_j diag(coef_j)
void filter_accum(hipStream_t st, int ne, int n, int m, const zd* E, const zd* coef, const zd* Y, const zd* rho, zd* Q,
                  bool add);
// the same with conjugation-closed columns: E holds the upper nodes' solutions
// only, node j's lower partner adds cl_j[c] conj(E_j[:, cp[c]]) to column c
void filter_accum_pair(hipStream_t st, int ne, int n, int m, const zd* E, const zd* cu, const zd* cl, const int* cp,
                       const zd* Y, const zd* rho, zd* Q, bool add);
// *flag_dev |= 1 when some entry of X (len) has a nonzero imaginary part
void any_imag(hipStream_t st, long len, const zd* X, int* flag_dev);
void ritz_residual(hipStream_t st, const CsrDev& A, bool conj_t, int n, int m, const zd* lam, bool conj_lam,
                   const zd* X, zd* Out);
void jacobi_diag(hipStream_t st, const SparseState& S, int ne, const zd* mvals, zd* jd);
void invert_vals(hipStream_t st, long len, zd* v);
template <typename T>
void scale_inplace(hipStream_t st, int n, int m, int nsys, Cx<T>* X, const double* sc);
template <typename T>
void add_same(hipStream_t st, long len, const Cx<T>* Z, Cx<T>* X);
void gather_vals(hipStream_t st, long len, bool complex_vals, const void* src, const int* idx, void* dst);
void cast_vals(hipStream_t st, long len, bool complex_vals, const void* src, void* dst);

}  // namespace fh
