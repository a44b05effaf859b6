// Grouped dense kernels: LU with partial pivoting and the 'N' / 'C' solves of
// many matrices of different sizes at once (every node of every instance of
// a batch), in FP64 or in complex FP32 whose GEMM updates run on MFMA.
// Each factorization / solve is precomputed into a plan of launches whose
// per-launch work lists live in one device buffer, so that the launch
// sequence is fixed and can be replayed or captured into a HIP graph.
#pragma once
#include "fh_kernels.h"

namespace fh {

constexpr int GNB = 32;   // panel / block width of the grouped LU and solves

// one GEMM of a grouped launch: C = (beta1 ? C : 0) + alpha op(A) B, row-major
template <typename T>
struct GItem {
    const Cx<T>* A;
    const Cx<T>* B;
    Cx<T>* C;
    int M, N, K, lda, ldb, ldc;
    int tiles_n, tile0;     // tiles along N; first tile index of this item
    Cx<T> alpha;
    int beta1;
};

// per-matrix entry of a panel / triangular-block launch
template <typename T>
struct GMat {
    Cx<T>* M;        // matrix (row-major, ld n)
    int* ipiv;       // n pivots (0-based)
    int* info;       // 0 or first zero pivot + 1
    Cx<T>* X;        // right-hand sides (n x m, ld m) for solves
    int n, k, jb;    // size, block start, block width
    int m;           // solves: right-hand-side columns of this matrix
};

enum GOpKind { GOP_PANEL, GOP_TRSM_ROW, GOP_GEMM_N, GOP_GEMM_C, GOP_LASWP_F, GOP_LASWP_R, GOP_DIAG };

struct GOp {
    int kind;
    int diag_variant;   // GOP_DIAG: 0 L (unit lower), 1 U (upper), 2 U^H (lower), 3 L^H (unit upper)
    size_t off;         // byte offset of the work list in the plan buffer
    int count;          // matrices or items
    int tiles;          // GEMM: total tiles; TRSM_ROW: column tiles of the largest matrix
    int mcols;          // solves: largest right-hand-side column count of the list
    double flops = 0.0; // GEMM: algorithmic flops (8 M N K per complex product)
    double bytes = 0.0; // GEMM: algorithmic bytes (A, B read, C read and written once)
    int narrow = 0;     // FP64 GEMM: 128 x 32 tiles (every item has at most 32 columns)
};

// GEMM tile used by the grouped MFMA kernel (chosen by the autotuner)
enum { GTILE_64 = 0, GTILE_32 = 1 };

template <typename T>
struct GroupPlan {
    std::vector<GOp> ops;
    DBuf buf;           // work lists
    int tile = GTILE_64;
    void run(hipStream_t st) const;
};

// factorization plan for matrices M[i] (n[i] x n[i]); ipiv[i], info[i] outputs
template <typename T>
void group_lu_plan(GroupPlan<T>& plan, int count, Cx<T>* const* M, const int* n, int* const* ipiv,
                   int* const* info, int tile);
// solve plan: op(M_i) X_i = X_i, X_i n[i] x m[i] (ld m[i]), op 'N' or 'C'
template <typename T>
void group_solve_plan(GroupPlan<T>& plan, char op, int count, Cx<T>* const* M, const int* n, int* const* ipiv,
                      Cx<T>* const* X, const int* m, int tile);
// grouped GEMM plan from explicit items (same conjugation for all)
template <typename T>
void group_gemm_plan(GroupPlan<T>& plan, bool conjA, std::vector<GItem<T>> items, int tile);

// elementwise helpers over a set of blocks (off/len/n/m/z: device arrays)
void set_resid_init(hipStream_t st, int count, int maxlen, const long* off, const int* len, const zd* z, const zd* Bv,
                    const zd* X, zd* R);
void set_colnorm(hipStream_t st, int count, int mmax, const long* off, const int* n, const int* m, const zd* V,
                 double* out);
void add_cast(hipStream_t st, long len, const cf* x, zd* y);
// X_s = identity for the count blocks (n[s] x n[s] at element offset off[s],
// device arrays); X must be zero on entry
void set_identity(hipStream_t st, int count, int nmax, const long* off, const int* n, cf* X);

}  // namespace fh
