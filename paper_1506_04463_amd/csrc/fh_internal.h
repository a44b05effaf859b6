// Internal state of handles and prepared problems.
#pragma once
#include <complex>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/feasthip.h"
#include "fh_kernels.h"
#include "fh_prof.h"

namespace fh {

struct SparseState;   // k_sparse.hip / sparse.cpp
struct NetState;      // k_net.hip / net.cpp
struct DenseGroup;    // k_group.hip / dgroup.cpp

struct FilterBufs {
    DBuf X, Xh, R, Rh, wdev, zdev;
};
struct FeastBufs {
    DBuf Ycur, Yhcur, Q, Qh, U, Uh, T1, T2, T3, T4, BQ, S, Sh, gam, AUr, BUr, lam, W, Wh, num, den, num2, den2,
        ints, perm;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    MemSourceP mem;   // caller's allocator (null: hipMalloc / hipFree)
    // scratch shared by the steps of one call
    DBuf eig_work, partial, partial2, small_i;
    FilterBufs fb;
    FeastBufs sb;
    bool prof_on = false;
    Prof prof;
    // autotuned grouped-GEMM tiles per shape class, and their probe scratch
    std::map<std::string, int> tuned;
    DBuf tune_scratch;
    // stream and events for HIP-graph capture and replay (created on first use)
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    ~Ctx() {
        if (gev[0]) (void)hipEventDestroy(gev[0]);
        if (gev[1]) (void)hipEventDestroy(gev[1]);
        if (gstream) (void)hipStreamDestroy(gstream);
    }
};

// makes the handle's profiler and memory source current on this thread for
// the duration of a call
struct ProfScope {
    MemScope mem;
    ProfScope(Ctx& c) : mem(c.mem, (void*)c.stream) { tl_prof() = c.prof_on ? &c.prof : nullptr; }
    ~ProfScope() { tl_prof() = nullptr; }
};

struct Prob {
    Ctx* h = nullptr;
    int n = 0;
    bool dense = true;
    fh_mat A{};
    fh_mat B{};
    bool hasB = false;
    // dense: cached LU of (z_j B - A) for the node set fact_z
    std::vector<std::complex<double>> fact_z;
    DBuf lu, ipiv, info;
    // dense grouped factors (complex-FP32 path)
    DenseGroup* dg = nullptr;
    // sparse state (CSR)
    SparseState* sp = nullptr;
    ~Prob();
};

using cplx = std::complex<double>;

// driver.cpp
// cpart (sparse problems with conj_pairs = 2): host array of m0 column
// partners, an involution, with Y[:, cpart[i]] = conj(Y[:, i]), the same for
// Yh, and lam[cpart[i]] = conj(lam[i]); the filter then solves the upper
// nodes' systems only.  nullptr: no such promise.
void filter(Ctx& c, Prob& p, int ne, const cplx* z, const cplx* w, int m0, const zd* Y, const zd* Yh, zd* Q,
            zd* Qh, const fh_opts& o, fh_report* rep, const cplx* lam = nullptr, const int* cpart = nullptr);
int feast(Ctx& c, Prob& p, const fh_contour& ct, const cplx* z, const cplx* w, const fh_opts& o, zd* Y, zd* Yh,
          zd* lambda, double* res, fh_report* rep);
void apply_A(Ctx& c, Prob& p, int side, int m, const zd* X, zd* Out);
void apply_B(Ctx& c, Prob& p, int side, int m, const zd* X, zd* Out);
void contour_nodes(const fh_contour& ct, std::vector<cplx>& z, std::vector<cplx>& w);

// sparse.cpp
void sparse_prepare(Ctx& c, Prob& p);
void sparse_filter(Ctx& c, Prob& p, int ne, const cplx* z, const cplx* w, int m0, const zd* Y, const zd* Yh,
                   zd* Q, zd* Qh, const fh_opts& o, fh_report* rep, const cplx* lam, const int* cpart = nullptr);
// true when conj_pairs = 2 applies to a FEAST run on this problem: a CSR
// matrix with real values and nodes that pair up as conjugates
bool sparse_conj_closed(const Prob& p, int ne, const cplx* z, const cplx* w, const fh_opts& o);
void sparse_apply_A(Ctx& c, Prob& p, int side, int m, const zd* X, zd* Out);
void sparse_shifted_apply(Ctx& c, Prob& p, int side, int nsys, const cplx* shifts, int m, const zd* X, zd* Out);
void sparse_residual_pair(Ctx& c, Prob& p, int side, int nsys, const cplx* shifts, int m, const zd* B, const zd* X,
                          const zd* Xt, zd* R, zd* E);
void sparse_ilu0(Ctx& c, Prob& p, cplx z, zd* lu_out);
void sparse_ilu0_apply(Ctx& c, Prob& p, cplx z, int side, int m, const zd* X, zd* Out);
void sparse_ilu0_apply32(Ctx& c, Prob& p, cplx z, int side, int m, const cf* X, cf* Out);
void sparse_destroy(SparseState* s);
void sparse_shifted_solve(Ctx& c, Prob& p, int nsys, const cplx* z, const int* sides, int m, const zd* B, zd* X,
                          const fh_opts& o, fh_report* rep);
void sparse_set_net(Prob& p, NetState* net);
void dg_destroy(DenseGroup* g);
void dense_filter_group(Ctx& c, Prob& p, int ne, const cplx* z, const cplx* w, int m0, const zd* Y, const zd* Yh,
                        zd* Q, zd* Qh, const fh_opts& o, fh_report* rep);
int feast_batched(Ctx& c, int count, Prob* const* probs, const fh_contour* cts, const fh_opts& o, zd* const* Y,
                  zd* const* Yh, zd* const* lambda, double* const* res, fh_report* reps);
void dense_shifted_solve(Ctx& c, Prob& p, int nsys, int nright, const cplx* z, int m, const zd* B, zd* X,
                         const fh_opts& o, fh_report* rep);

// net.cpp
NetState* net_create(Ctx& c, int nz, int ny, int nx, int nfields, const double* fields, double alpha,
                     double out_scale, unsigned long long seed);
void net_destroy(NetState* s);
int net_param_count(const NetState* s);
int net_grid_size(const NetState* s);
void net_set_params(Ctx& c, NetState& S, const float* host);
void net_set_fields(Ctx& c, NetState& S, const double* fields);
void net_set_activations(NetState& S, int bf16);
int net_field_count(const NetState* s);
void net_get_params(Ctx& c, NetState& S, float* host);
void net_forward_host(Ctx& c, NetState& S, int nsys, int m, const zd* X, const double* shifts, const int* sides, zd* Out);
double net_loss_grad(Ctx& c, NetState& S, const SparseState* sp, int nsys, int m, const zd* R, const zd* E,
                     const double* shifts, const int* sides, bool step, double lr);
void net_get_grad(Ctx& c, NetState& S, float* host);

}  // namespace fh
