// extern "C" entry points of include/feasthip.h: argument checks, error
// capture, dispatch to the driver.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <mutex>

#include "fh_internal.h"

using namespace fh;

struct fh_ctx : Ctx {};
struct fh_prob : Prob {};
struct fh_net_s {
    NetState* st = nullptr;
    int device = 0;
    ~fh_net_s() {
        if (st) net_destroy(st);
    }
};

namespace fh {
Prob::~Prob() {
    if (sp) sparse_destroy(sp);
    sp = nullptr;
    if (dg) dg_destroy(dg);
    dg = nullptr;
}
}  // namespace fh

#define FH_API_BEGIN(hh) \
    try {                    \
        ProfScope prof_scope_(*(hh));
#define FH_API_END(hh)                                        \
    }                                                         \
    catch (const fh::Error& e) {                              \
        if (hh) (hh)->err = e.what();                         \
        return e.code;                                        \
    }                                                         \
    catch (const std::exception& e) {                         \
        if (hh) (hh)->err = e.what();                         \
        return FH_HIP_ERROR;                                  \
    }

static void set_device(Ctx* c) { FH_HIP(hipSetDevice(c->device)); }

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free entry point (fh_reduced_matrix_noalloc):
// one static array per device, resolved to its device address once per device
// in fh_create.  Host code uses only the resolved addresses, never the array's
// name.
// ---------------------------------------------------------------------------
static constexpr size_t kScratchBytes = size_t(FH_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static int resolve_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return FH_HIP_ERROR;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return FH_OK;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return FH_HIP_ERROR;
    if (hipSetDevice(device) != hipSuccess) return FH_HIP_ERROR;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || ptr == nullptr) return FH_HIP_ERROR;
    g_scratch_ptr[device] = ptr;
    return FH_OK;
}

static void* scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

extern "C" {

void fh_default_opts(fh_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->m0 = 0;
    o->max_iter = 50;
    o->eps = 1e-12;
    o->precision = FH_PREC_FP64;
    o->solver = FH_SOLVER_LU;
    o->restart = 30;
    o->block = 0;
    o->precond = FH_PC_ILU0;
    o->inner_tol = 1e-12;
    o->max_restarts = 50;
    o->mixed_inner_tol = 1e-5;
    o->max_refine = 8;
    o->save_factors = 1;
    o->resume = 0;
    o->fallback = FH_PC_ILU0;
    o->graph = 0;
    o->orth = 0;
    o->batch_nodes = 0;
    o->sym = 0;
    o->confirm = 0;
    o->conj_pairs = 1;
}

int fh_create(fh_handle* h, int device, void* stream, const fh_allocator* alloc) {
    if (!h) return -1;
    *h = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FH_HIP_ERROR;
    if (device < 0 || device >= ndev) return -2;
    if (alloc && (!alloc->alloc || !alloc->free)) return -4;
    if (resolve_scratch(device) != FH_OK) return FH_HIP_ERROR;
    fh_ctx* c = new fh_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    if (alloc) {
        c->mem = std::make_shared<MemSource>();
        c->mem->alloc = alloc->alloc;
        c->mem->free = alloc->free;
        c->mem->user = alloc->user;
    }
    *h = c;
    return FH_OK;
}

int fh_profile(fh_handle h, int enable) {
    if (!h) return -1;
    FH_API_BEGIN(h)
    h->prof.reset();
    h->prof_on = enable != 0;
    return FH_OK;
    FH_API_END(h)
}

int fh_profile_read(fh_handle h, int idx, char* name, int namelen, long long* count, double* ms, double* bytes,
                    double* flops) {
    if (!h) return -1;
    if (idx < 0) return -2;
    if (!name || namelen < 1) return -3;
    FH_API_BEGIN(h)
    h->prof.resolve();
    if (idx >= (int)h->prof.stats.size()) return 1;
    auto it = h->prof.stats.begin();
    std::advance(it, idx);
    std::snprintf(name, namelen, "%s", it->first.c_str());
    if (count) *count = it->second.count;
    if (ms) *ms = it->second.ms;
    if (bytes) *bytes = it->second.bytes;
    if (flops) *flops = it->second.flops;
    return FH_OK;
    FH_API_END(h)
}

int fh_destroy(fh_handle h) {
    if (!h) return -1;
    delete h;
    return FH_OK;
}

int fh_set_stream(fh_handle h, void* stream) {
    if (!h) return -1;
    h->stream = (hipStream_t)stream;
    return FH_OK;
}

const char* fh_last_error(fh_handle h) { return h ? h->err.c_str() : "null handle"; }

// an ellipse with positive axes, or a polygon of nv >= 3 vertices whose node
// count is a positive multiple of nv
static bool contour_ok(const fh_contour& c) {
    if (c.ne < 1) return false;
    if (c.nv == 0) return c.a > 0 && c.ratio > 0;
    return c.nv >= 3 && c.verts != nullptr && c.ne % c.nv == 0;
}

int fh_contour_nodes(const fh_contour* c, double* z, double* w) {
    if (!c) return -1;
    if (!z) return -2;
    if (!w) return -3;
    if (!contour_ok(*c)) return -1;
    std::vector<cplx> zz, ww;
    contour_nodes(*c, zz, ww);
    std::memcpy(z, zz.data(), sizeof(cplx) * c->ne);
    std::memcpy(w, ww.data(), sizeof(cplx) * c->ne);
    return FH_OK;
}

int fh_rational(int ne, const double* z, const double* w, int nlam, const double* lam, double* rho) {
    if (ne < 1) return -1;
    if (!z) return -2;
    if (!w) return -3;
    if (nlam < 0) return -4;
    if (nlam > 0 && !lam) return -5;
    if (nlam > 0 && !rho) return -6;
    const cplx* zc = reinterpret_cast<const cplx*>(z);
    const cplx* wc = reinterpret_cast<const cplx*>(w);
    const cplx* lc = reinterpret_cast<const cplx*>(lam);
    cplx* rc = reinterpret_cast<cplx*>(rho);
    for (int i = 0; i < nlam; ++i) {
        cplx s = 0.0;
        for (int j = 0; j < ne; ++j) s += wc[j] / (zc[j] - lc[i]);
        rc[i] = s;
    }
    return FH_OK;
}

int fh_problem_create(fh_handle h, const fh_mat* A, const fh_mat* B, fh_problem* out) {
    if (!h) return -1;
    if (!A) return -2;
    if (!out) return -4;
    *out = nullptr;
    FH_API_BEGIN(h)
    set_device(h);
    if (A->n <= 0) return -2;
    if (A->kind == FH_DENSE) {
        if (A->dtype != FH_C128 || !A->val || A->ld < A->n) return -2;
        if (B && (B->kind != FH_DENSE || B->dtype != FH_C128 || B->n != A->n || !B->val || B->ld < B->n)) return -3;
    } else if (A->kind == FH_CSR) {
        if ((A->dtype != FH_R64 && A->dtype != FH_C128) || !A->val || !A->rowptr || !A->colind || A->nnz < A->n)
            return -2;
        if (B) return -3;   // sparse problems take B = I
    } else {
        return -2;
    }
    fh_prob* p = new fh_prob();
    p->h = h;
    p->n = A->n;
    p->A = *A;
    p->dense = (A->kind == FH_DENSE);
    p->hasB = (B != nullptr);
    if (B) p->B = *B;
    try {
        if (!p->dense) sparse_prepare(*h, *p);
    } catch (...) {
        delete p;
        throw;
    }
    *out = p;
    return FH_OK;
    FH_API_END(h)
}

int fh_problem_destroy(fh_problem p) {
    if (!p) return -1;
    delete p;
    return FH_OK;
}

static int check_opts(const fh_opts* o, int m0, int n) {
    if (!o) return 0;
    if (m0 < 1 || m0 > n || m0 > 1024) return 1;
    return 0;
}

int fh_filter(fh_handle h, fh_problem p, int ne, const double* z, const double* w, int m0, const void* Y,
              const void* Yh, void* Q, void* Qh, const fh_opts* o, fh_report* rep) {
    if (!h) return -1;
    if (!p) return -2;
    if (ne < 1) return -3;
    if (!z) return -4;
    if (!w) return -5;
    if (m0 < 1 || m0 > p->n || m0 > 1024) return -6;
    if (!Y) return -7;
    if (!Yh) return -8;
    if (!Q) return -9;
    if (!Qh) return -10;
    fh_opts def;
    fh_default_opts(&def);
    def.m0 = m0;
    if (!o) { o = &def; if (!p->dense) def.solver = FH_SOLVER_BGMRES; }
    FH_API_BEGIN(h)
    set_device(h);
    fh_report local{};
    fh_report* r = rep ? rep : &local;
    std::memset(r, 0, sizeof(*r));
    filter(*h, *p, ne, reinterpret_cast<const cplx*>(z), reinterpret_cast<const cplx*>(w), m0, (const zd*)Y,
           (const zd*)Yh, (zd*)Q, (zd*)Qh, *o, r);
    r->info = FH_OK;
    return FH_OK;
    FH_API_END(h)
}

int fh_feast(fh_handle h, fh_problem p, const fh_contour* c, const double* z, const double* w, const fh_opts* o,
             void* Y, void* Yh, void* lambda, double* res, fh_report* rep) {
    if (!h) return -1;
    if (!p) return -2;
    if (!c || !contour_ok(*c)) return -3;
    if ((z == nullptr) != (w == nullptr)) return -4;
    if (!o) return -6;
    if (o->m0 < 1 || o->m0 > p->n || o->m0 > 1024 || o->max_iter < 1 || !(o->eps > 0)) return -6;
    if (!Y) return -7;
    if (!Yh) return -8;
    if (!lambda) return -9;
    FH_API_BEGIN(h)
    set_device(h);
    fh_report local{};
    fh_report* r = rep ? rep : &local;
    std::memset(r, 0, sizeof(*r));
    int info = feast(*h, *p, *c, reinterpret_cast<const cplx*>(z), reinterpret_cast<const cplx*>(w), *o, (zd*)Y,
                     (zd*)Yh, (zd*)lambda, res, r);
    r->info = info;
    return info;
    FH_API_END(h)
}

int fh_count_estimate(fh_handle h, fh_problem p, int ne, const double* z, const double* w, int nprobe,
                      const void* V, const fh_opts* o, double* est, fh_report* rep) {
    if (!h) return -1;
    if (!p) return -2;
    if (ne < 1) return -3;
    if (!z) return -4;
    if (!w) return -5;
    if (nprobe < 1 || nprobe > 256 || nprobe > p->n) return -6;
    if (!V) return -7;
    if (!est) return -9;
    fh_opts def;
    fh_default_opts(&def);
    def.m0 = nprobe;
    if (!o) { o = &def; if (!p->dense) def.solver = FH_SOLVER_BGMRES; }
    FH_API_BEGIN(h)
    set_device(h);
    fh_report local{};
    fh_report* r = rep ? rep : &local;
    std::memset(r, 0, sizeof(*r));
    const size_t blk = (size_t)p->n * nprobe;
    DBuf qb, hb, cb;
    zd* Q = (zd*)qb.ensure(sizeof(zd) * blk);
    // sparse problems: right solves only (no left block); dense: the filter's
    // left half runs on the probes too and is discarded
    zd* Qh = p->dense ? (zd*)hb.ensure(sizeof(zd) * blk) : nullptr;
    const zd* Yh = p->dense ? (const zd*)V : nullptr;
    filter(*h, *p, ne, reinterpret_cast<const cplx*>(z), reinterpret_cast<const cplx*>(w), nprobe, (const zd*)V, Yh,
           Q, Qh, *o, r);
    zd* C = (zd*)cb.ensure(sizeof(zd) * (size_t)nprobe * nprobe);
    gemm_hn_tall(h->stream, p->n, nprobe, nprobe, (const zd*)V, nprobe, Q, nprobe, C, nprobe, h->partial);
    std::vector<zd> hc((size_t)nprobe * nprobe);
    FH_HIP(hipMemcpyAsync(hc.data(), C, sizeof(zd) * hc.size(), hipMemcpyDeviceToHost, h->stream));
    FH_HIP(hipStreamSynchronize(h->stream));
    double re = 0.0, im = 0.0;
    for (int k = 0; k < nprobe; ++k) {
        re += hc[(size_t)k * nprobe + k].re;
        im += hc[(size_t)k * nprobe + k].im;
    }
    est[0] = re / nprobe;
    est[1] = im / nprobe;
    r->info = FH_OK;
    return FH_OK;
    FH_API_END(h)
}

int fh_reduced_matrix(fh_handle h, fh_problem p, int m, const void* Qh, const void* Q, void* BQ) {
    if (!h) return -1;
    if (!p) return -2;
    if (m < 1) return -3;
    if (!Qh) return -4;
    if (!Q) return -5;
    if (!BQ) return -6;
    FH_API_BEGIN(h)
    set_device(h);
    DBuf tmp;
    const zd* Bq = (const zd*)Q;
    if (p->hasB) {
        zd* t = (zd*)tmp.ensure(sizeof(zd) * (size_t)p->n * m);
        apply_B(*h, *p, 0, m, (const zd*)Q, t);
        Bq = t;
    }
    gemm_hn_tall(h->stream, p->n, m, m, (const zd*)Qh, m, Bq, m, (zd*)BQ, m, h->partial);
    FH_HIP(hipStreamSynchronize(h->stream));
    return FH_OK;
    FH_API_END(h)
}

int fh_reduced_matrix_noalloc(fh_handle h, fh_problem p, int m, const void* Qh, const void* Q, void* BQ) {
    if (!h) return -1;
    if (!p) return -2;
    if (m < 1) return -3;
    if (!Qh) return -4;
    if (!Q) return -5;
    if (!BQ) return -6;
    const size_t part_min = sizeof(zd) * (size_t)m * m;         // one partial m x m block
    const size_t bq_tmp = p->hasB ? sizeof(zd) * (size_t)p->n * m : 0;   // B Q
    if (bq_tmp + part_min > kScratchBytes) {
        h->err = "fh_reduced_matrix_noalloc: needs " + std::to_string(bq_tmp + part_min) +
                 " bytes of scratch (m^2 * 16, plus n * m * 16 with a B matrix), more than its " +
                 std::to_string(kScratchBytes);
        return -3;
    }
    try {
        FH_HIP(hipSetDevice(h->device));
        unsigned char* base = (unsigned char*)scratch_of(h->device);
        FH_REQUIRE(base != nullptr, FH_HIP_ERROR, "fh_reduced_matrix_noalloc: scratch not resolved for this device");
        const zd* Bq = (const zd*)Q;
        if (p->hasB) {
            zd* t = (zd*)base;
            apply_B(*h, *p, 0, m, (const zd*)Q, t);
            Bq = t;
        }
        const size_t off = (bq_tmp + 255) / 256 * 256;
        const bool ok = gemm_hn_tall_into(h->stream, p->n, m, m, (const zd*)Qh, m, Bq, m, (zd*)BQ, m, base + off,
                                          kScratchBytes - off);
        FH_REQUIRE(ok, -3, "fh_reduced_matrix_noalloc: m too large for the scratch");
        FH_HIP(hipStreamSynchronize(h->stream));
        return FH_OK;
    } catch (const fh::Error& e) {
        h->err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        h->err = e.what();
        return FH_HIP_ERROR;
    }
}

int fh_biortho_factors(fh_handle h, int m, const void* BQ, double eta, void* gamma, void* S, void* Sh, int* m0t) {
    if (!h) return -1;
    if (m < 1 || m > 1024) return -2;
    if (!BQ) return -3;
    if (!(eta >= 0)) return -4;
    if (!gamma) return -5;
    if (!S) return -6;
    if (!Sh) return -7;
    if (!m0t) return -8;
    FH_API_BEGIN(h)
    set_device(h);
    int* d = (int*)h->small_i.ensure(sizeof(int) * 4);
    eig_biortho(h->stream, m, (const zd*)BQ, eta, (zd*)gamma, (zd*)S, (zd*)Sh, d, d + 1, h->eig_work);
    int hv[2];
    FH_HIP(hipMemcpyAsync(hv, d, sizeof(hv), hipMemcpyDeviceToHost, h->stream));
    FH_HIP(hipStreamSynchronize(h->stream));
    *m0t = hv[0];
    if (hv[1] != 0) throw Error(FH_EIG_FAILED, "eigendecomposition of B_Q failed");
    return FH_OK;
    FH_API_END(h)
}

int fh_reduced_eig(fh_handle h, int m, const void* AU, const void* BU, void* lambda, void* W, void* Wh) {
    if (!h) return -1;
    if (m < 1 || m > 1024) return -2;
    if (!AU) return -3;
    if (!BU) return -4;
    if (!lambda) return -5;
    if (!W) return -6;
    if (!Wh) return -7;
    FH_API_BEGIN(h)
    set_device(h);
    int* d = (int*)h->small_i.ensure(sizeof(int) * 4);
    eig_reduced(h->stream, m, (const zd*)AU, (const zd*)BU, (zd*)lambda, (zd*)W, (zd*)Wh, d, h->eig_work);
    int hv = 0;
    FH_HIP(hipMemcpyAsync(&hv, d, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    FH_HIP(hipStreamSynchronize(h->stream));
    if (hv != 0) throw Error(FH_EIG_FAILED, "reduced eigenproblem failed");
    return FH_OK;
    FH_API_END(h)
}

int fh_shifted_apply(fh_handle h, fh_problem p, int side, int nsys, const double* shifts, int m, const void* X,
                     void* Out) {
    if (!h) return -1;
    if (!p) return -2;
    if (side != 0 && side != 1) return -3;
    if (nsys < 1) return -4;
    if (!shifts) return -5;
    if (m < 1) return -6;
    if (!X) return -7;
    if (!Out) return -8;
    FH_API_BEGIN(h)
    set_device(h);
    const cplx* s = reinterpret_cast<const cplx*>(shifts);
    if (p->dense) {
        const size_t blk = (size_t)p->n * m;
        for (int k = 0; k < nsys; ++k) {
            zd* o = (zd*)Out + k * blk;
            const zd* x = (const zd*)X + k * blk;
            apply_A(*h, *p, side, m, x, o);
            const cplx sh = s[k];
            shift_combine(h->stream, (long)blk, cx(sh.real(), sh.imag()), x, o);   // o = sh x - A x
        }
    } else {
        sparse_shifted_apply(*h, *p, side, nsys, s, m, (const zd*)X, (zd*)Out);
    }
    FH_HIP(hipStreamSynchronize(h->stream));
    return FH_OK;
    FH_API_END(h)
}

int fh_residual_pair(fh_handle h, fh_problem p, int side, int nsys, const double* shifts, int m, const void* B,
                     const void* X, const void* Xt, void* R, void* E) {
    if (!h) return -1;
    if (!p || p->dense) return -2;
    if (side != 0 && side != 1) return -3;
    if (nsys < 1) return -4;
    if (!shifts) return -5;
    if (m < 1) return -6;
    if (!B) return -7;
    if (!X) return -8;
    if (!Xt) return -9;
    if (!R) return -10;
    if (!E) return -11;
    FH_API_BEGIN(h)
    set_device(h);
    sparse_residual_pair(*h, *p, side, nsys, reinterpret_cast<const cplx*>(shifts), m, (const zd*)B, (const zd*)X,
                         (const zd*)Xt, (zd*)R, (zd*)E);
    return FH_OK;
    FH_API_END(h)
}

int fh_ilu0(fh_handle h, fh_problem p, double z_re, double z_im, void* lu) {
    if (!h) return -1;
    if (!p || p->dense) return -2;
    if (!lu) return -5;
    FH_API_BEGIN(h)
    set_device(h);
    sparse_ilu0(*h, *p, cplx(z_re, z_im), (zd*)lu);
    FH_HIP(hipStreamSynchronize(h->stream));
    return FH_OK;
    FH_API_END(h)
}

int fh_ilu0_apply(fh_handle h, fh_problem p, double z_re, double z_im, int side, int m, const void* X, void* Out) {
    if (!h) return -1;
    if (!p || p->dense) return -2;
    if (side != 0 && side != 1) return -5;
    if (m < 1) return -6;
    if (!X) return -7;
    if (!Out) return -8;
    FH_API_BEGIN(h)
    set_device(h);
    sparse_ilu0_apply(*h, *p, cplx(z_re, z_im), side, m, (const zd*)X, (zd*)Out);
    FH_HIP(hipStreamSynchronize(h->stream));
    return FH_OK;
    FH_API_END(h)
}

int fh_ilu0_apply_c64(fh_handle h, fh_problem p, double z_re, double z_im, int side, int m, const void* X,
                      void* Out) {
    if (!h) return -1;
    if (!p || p->dense) return -2;
    if (side != 0 && side != 1) return -5;
    if (m < 1) return -6;
    if (!X) return -7;
    if (!Out) return -8;
    FH_API_BEGIN(h)
    set_device(h);
    sparse_ilu0_apply32(*h, *p, cplx(z_re, z_im), side, m, (const cf*)X, (cf*)Out);
    FH_HIP(hipStreamSynchronize(h->stream));
    return FH_OK;
    FH_API_END(h)
}

int fh_feast_batched(fh_handle h, int count, const fh_problem* problems, const fh_contour* contours,
                     const fh_opts* o, void* const* Y, void* const* Yh, void* const* lambda, double* const* res,
                     fh_report* reports) {
    if (!h) return -1;
    if (count < 1) return -2;
    if (!problems) return -3;
    if (!contours) return -4;
    if (!o || o->m0 < 1 || o->m0 > 1024 || o->max_iter < 1 || !(o->eps > 0)) return -5;
    if (o->precision != FH_PREC_FP64 && o->precision != FH_PREC_MIXED) return -5;
    if (!Y) return -6;
    if (!Yh) return -7;
    if (!lambda) return -8;
    for (int i = 0; i < count; ++i) {
        if (!problems[i] || !problems[i]->dense || o->m0 > problems[i]->n) return -3;
        const fh_contour& c = contours[i];
        if (!contour_ok(c)) return -4;
        if (!Y[i]) return -6;
        if (!Yh[i]) return -7;
        if (!lambda[i]) return -8;
    }
    FH_API_BEGIN(h)
    set_device(h);
    std::vector<Prob*> ps(count);
    std::vector<zd*> y(count), yh(count), l(count);
    std::vector<double*> r(count, nullptr);
    for (int i = 0; i < count; ++i) {
        ps[i] = problems[i];
        y[i] = (zd*)Y[i];
        yh[i] = (zd*)Yh[i];
        l[i] = (zd*)lambda[i];
        if (res) r[i] = res[i];
    }
    return feast_batched(*h, count, ps.data(), contours, *o, y.data(), yh.data(), l.data(), r.data(), reports);
    FH_API_END(h)
}

int fh_shifted_solve(fh_handle h, fh_problem p, int nsys, const double* z, const int* sides, int m,
                     const fh_opts* o, const void* B, void* X, fh_report* rep) {
    if (!h) return -1;
    if (!p) return -2;
    if (nsys < 1) return -3;
    if (!z) return -4;
    if (!sides) return -5;
    if (m < 1 || (!p->dense && m > 256)) return -6;
    if (!o) return -7;
    if (!B) return -8;
    if (!X) return -9;
    int nright = 0;
    while (nright < nsys && sides[nright] == 0) ++nright;
    for (int s = nright; s < nsys; ++s)
        if (sides[s] != 1) return -5;
    if (o->precision != FH_PREC_FP64 && o->precision != FH_PREC_MIXED) return -7;
    if (o->precond < FH_PC_NONE || o->precond > FH_PC_LEARNED) return -7;
    if (o->precond == FH_PC_LEARNED && (o->fallback < FH_PC_NONE || o->fallback > FH_PC_ILU0)) return -7;
    FH_API_BEGIN(h)
    set_device(h);
    if (rep) std::memset(rep, 0, sizeof(*rep));
    const cplx* zc = reinterpret_cast<const cplx*>(z);
    if (p->dense)
        dense_shifted_solve(*h, *p, nsys, nright, zc, m, (const zd*)B, (zd*)X, *o, rep);
    else
        sparse_shifted_solve(*h, *p, nsys, zc, sides, m, (const zd*)B, (zd*)X, *o, rep);
    FH_HIP(hipStreamSynchronize(h->stream));
    return FH_OK;
    FH_API_END(h)
}

int fh_net_create(fh_handle h, int nz, int ny, int nx, int nfields, const double* fields, double alpha,
                  double out_scale, unsigned long long seed, fh_net* out) {
    if (!h) return -1;
    if (nz < 1) return -2;
    if (ny < 1) return -3;
    if (nx < 1) return -4;
    if (nfields < 0 || nfields > FH_NET_MAX_FIELDS) return -5;
    if (nfields > 0 && !fields) return -6;
    if (!(alpha > 0)) return -7;
    if (!(out_scale > 0)) return -8;
    if (!out) return -10;
    *out = nullptr;
    FH_API_BEGIN(h)
    set_device(h);
    fh_net_s* n = new fh_net_s();
    n->device = h->device;
    try {
        n->st = net_create(*h, nz, ny, nx, nfields, fields, alpha, out_scale, seed);
    } catch (...) {
        delete n;
        throw;
    }
    *out = n;
    return FH_OK;
    FH_API_END(h)
}

int fh_net_destroy(fh_net net) {
    if (!net) return -1;
    (void)hipSetDevice(net->device);
    delete net;
    return FH_OK;
}

int fh_net_param_count(fh_net net) {
    if (!net) return -1;
    return net_param_count(net->st);
}

int fh_net_get_params(fh_handle h, fh_net net, float* params) {
    if (!h) return -1;
    if (!net) return -2;
    if (!params) return -3;
    FH_API_BEGIN(h)
    set_device(h);
    net_get_params(*h, *net->st, params);
    return FH_OK;
    FH_API_END(h)
}

int fh_net_set_params(fh_handle h, fh_net net, const float* params) {
    if (!h) return -1;
    if (!net) return -2;
    if (!params) return -3;
    FH_API_BEGIN(h)
    set_device(h);
    net_set_params(*h, *net->st, params);
    return FH_OK;
    FH_API_END(h)
}

// operator shift per system: z for a right system, conj(z) for a left one
static std::vector<double> op_shifts(int nsys, const double* z, const int* sides) {
    std::vector<double> s(2 * (size_t)nsys);
    for (int k = 0; k < nsys; ++k) {
        s[2 * k] = z[2 * k];
        s[2 * k + 1] = sides[k] ? -z[2 * k + 1] : z[2 * k + 1];
    }
    return s;
}

int fh_net_set_fields(fh_handle h, fh_net net, const double* fields) {
    if (!h) return -1;
    if (!net) return -2;
    if (!fields && net_field_count(net->st) > 0) return -3;
    FH_API_BEGIN(h)
    set_device(h);
    if (net_field_count(net->st) > 0) net_set_fields(*h, *net->st, fields);
    return FH_OK;
    FH_API_END(h)
}

int fh_net_set_activations(fh_net net, int bf16) {
    if (!net) return -1;
    if (bf16 != 0 && bf16 != 1) return -2;
    net_set_activations(*net->st, bf16);
    return FH_OK;
}

int fh_net_forward(fh_handle h, fh_net net, int nsys, int m, const double* z, const int* sides, const void* V,
                   void* Out) {
    if (!h) return -1;
    if (!net) return -2;
    if (nsys < 1) return -3;
    if (m < 1) return -4;
    if (!z) return -5;
    if (!sides) return -6;
    if (!V) return -7;
    if (!Out) return -8;
    for (int s = 0; s < nsys; ++s)
        if (sides[s] != 0 && sides[s] != 1) return -6;
    FH_API_BEGIN(h)
    set_device(h);
    std::vector<double> sh = op_shifts(nsys, z, sides);
    net_forward_host(*h, *net->st, nsys, m, (const zd*)V, sh.data(), sides, (zd*)Out);
    return FH_OK;
    FH_API_END(h)
}

int fh_net_train_step(fh_handle h, fh_net net, fh_problem p, int nsys, int m, const double* z, const int* sides,
                      const void* R, const void* E, double lr, int update, double* loss, float* grad) {
    if (!h) return -1;
    if (!net) return -2;
    if (p && (p->dense || p->n != net_grid_size(net->st))) return -3;
    if (nsys < 1) return -4;
    if (m < 1 || (p && m > 256)) return -5;
    if (!z) return -6;
    if (!sides) return -7;
    if (!R) return -8;
    if (!E) return -9;
    if (update && !(lr > 0)) return -10;
    for (int s = 0; s < nsys; ++s)
        if (sides[s] != 0 && sides[s] != 1) return -7;
    FH_API_BEGIN(h)
    set_device(h);
    std::vector<double> sh = op_shifts(nsys, z, sides);
    const double l = net_loss_grad(*h, *net->st, p ? p->sp : nullptr, nsys, m, (const zd*)R, (const zd*)E,
                                   sh.data(), sides, update != 0, lr);
    if (loss) *loss = l;
    if (grad) net_get_grad(*h, *net->st, grad);
    return FH_OK;
    FH_API_END(h)
}

int fh_problem_set_net(fh_problem p, fh_net net) {
    if (!p || p->dense) return -1;
    if (net && net_grid_size(net->st) != p->n) return -2;
    sparse_set_net(*p, net ? net->st : nullptr);
    return FH_OK;
}

}  // extern "C"
