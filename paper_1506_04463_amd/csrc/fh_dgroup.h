// Dense shifted systems (z_s B - A) of one or many problems solved together
// with the grouped kernels (Section 2.4: one factorization per node, reused
// for the right and the left solves): FP64 LU and direct solves, or a
// complex-FP32 LU (GEMM updates on MFMA) inside FP64 iterative refinement of
// every right-hand side.  In the complex-FP32 case the inverse of each
// factorization is formed once (LU X = I, grouped solves with n right-hand
// sides), so that every refinement step's solve is one grouped MFMA GEMM
// (d = M^{-1} r, d = M^{-H} r on the left) instead of a chain of dependent
// triangular-block launches; the FP64 residuals keep the refinement exact.
#pragma once
#include <complex>
#include <memory>

#include "fh_group.h"
#include "fh_internal.h"

namespace fh {

struct DenseGroup {
    bool mixed = false;
    int count = 0;                  // systems per side (one per (problem, node))
    std::vector<Prob*> prob;        // per system
    std::vector<int> n;             // per system
    std::vector<std::complex<double>> z;
    int tile_lu = GTILE_64, tile_solve = GTILE_32;
    // factors
    DBuf M64, M32, Inv32, ipiv, info, dz, dzc;
    std::vector<size_t> moff;       // element offset of each matrix
    std::vector<size_t> poff;       // pivot offset of each matrix
    // right-hand-side layout: block s is n[s] x m[s] (ld m[s]) at voff[s]
    std::vector<int> m;
    std::vector<long> voff;
    long vtot = 0;
    int mmax = 0, maxlen = 0;
    DBuf Bv, Bhv, Xv, Xhv, X32, Xh32, T32, Th32, R, Rh, doff, dlen, dn, dm, nrm;
    GroupPlan<double> sN64, sC64, resN, resC, resBN, resBC;
    GroupPlan<float> sN32, sC32;
    const void* layout_key[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    long layout_vtot = -1;
    // captured launch sequences (valid for the current layout)
    hipGraphExec_t g_fp64 = nullptr, g_first = nullptr, g_next = nullptr;
    DBuf zb;                        // shifts of the residual initialisation
    // complex-FP32 groups: FP64 factors of the systems whose refinement
    // stalled above the inner tolerance (built on demand, kept while the set
    // of such systems does not change)
    std::unique_ptr<DenseGroup> fb64;
    std::vector<int> fb_sys;
    void drop_graphs() {
        for (hipGraphExec_t* g : {&g_fp64, &g_first, &g_next})
            if (*g) {
                (void)hipGraphExecDestroy(*g);
                *g = nullptr;
            }
    }
    ~DenseGroup() { drop_graphs(); }
};

// Form and factor (z_s B_p - A_p) for the nodes zs[p] of every problem p.
void dg_build(Ctx& c, DenseGroup& G, const std::vector<Prob*>& probs,
              const std::vector<std::vector<std::complex<double>>>& zs, bool mixed, fh_report* rep);
// Set the right-hand-side counts (one per system) and (re)build the solve
// plans when the layout changes; afterwards G.Bv / G.Bhv hold the right /
// left right-hand sides and dg_solve leaves the solutions in G.Xv / G.Xhv.
void dg_layout(Ctx& c, DenseGroup& G, const std::vector<int>& m);
// Right solves (z_s B - A) X = B and left solves (z_s B - A)^H Xh = Bh of
// every system.  Mixed: refinement until the worst relative residual is at
// most o.inner_tol or o.max_refine steps; returns that residual (0 for FP64).
double dg_solve(Ctx& c, DenseGroup& G, const fh_opts& o, fh_report* rep);

}  // namespace fh
