#include "fh_internal.h"
namespace fh {
struct SparseState {};
static void nyi() { throw Error(FH_HIP_ERROR, "sparse path not built"); }
void sparse_prepare(Ctx&, Prob&) { nyi(); }
void sparse_filter(Ctx&, Prob&, int, const cplx*, const cplx*, int, const zd*, const zd*, zd*, zd*, const fh_opts&, fh_report*) { nyi(); }
void sparse_apply_A(Ctx&, Prob&, int, int, const zd*, zd*) { nyi(); }
void sparse_shifted_apply(Ctx&, Prob&, int, int, const cplx*, int, const zd*, zd*) { nyi(); }
void sparse_ilu0(Ctx&, Prob&, cplx, zd*) { nyi(); }
void sparse_ilu0_apply(Ctx&, Prob&, cplx, int, int, const zd*, zd*) { nyi(); }
void sparse_destroy(SparseState* s) { delete s; }
}
