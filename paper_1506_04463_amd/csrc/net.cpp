// Host side of the learned preconditioner: parameter layout and
// initialization, batched forward / loss / backward / Adam steps driven from
// the C ABI, and the preconditioner apply used by FGMRES.
#include <cmath>
#include <random>

#include "fh_net.h"
#include "fh_sparse.h"

namespace fh {

static void layout(NetDev& d) {
    const int T = d.taps;
    int off = 0;
    d.off_w1 = off; off += NET_HID * d.cin * T;
    d.off_b1 = off; off += NET_HID;
    d.off_w2 = off; off += NET_HID * NET_HID * T;
    d.off_b2 = off; off += NET_HID;
    d.off_w3 = off; off += 2 * NET_HID * T;
    d.off_b3 = off; off += 2;
    d.np = off;
}

NetState* net_create(Ctx& c, int nz, int ny, int nx, int nfields, const double* fields, double alpha,
                     double out_scale, unsigned long long seed) {
    FH_REQUIRE(nz > 0 && ny > 0 && nx > 0, -2, "network grid must be positive");
    FH_REQUIRE(nfields >= 0 && NET_FIXED_CH + nfields <= NET_MAX_CIN, -4, "too many input fields");
    NetState* S = new NetState();
    NetDev& d = S->d;
    d.nz = nz;
    d.ny = ny;
    d.nx = nx;
    d.taps = nz > 1 ? 27 : 9;
    d.cin = NET_FIXED_CH + nfields;
    d.inv_alpha = alpha > 0 ? 1.0 / alpha : 1.0;
    d.oscale = out_scale > 0 ? (float)out_scale : 1.0f;
    layout(d);
    // He-normal initialisation, zero biases, last layer scaled down
    std::vector<float> w(d.np, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    auto fill = [&](int off, int cnt, int fan_in, double gain) {
        const double s = gain * std::sqrt(2.0 / fan_in);
        for (int i = 0; i < cnt; ++i) w[off + i] = (float)(s * nd(rng));
    };
    const int T = d.taps;
    fill(d.off_w1, NET_HID * d.cin * T, d.cin * T, 1.0);
    fill(d.off_w2, NET_HID * NET_HID * T, NET_HID * T, 1.0);
    fill(d.off_w3, 2 * NET_HID * T, NET_HID * T, 0.1);
    d.w = (float*)S->w.ensure(sizeof(float) * d.np);
    d.wb = (uint16_t*)S->wb.ensure(sizeof(uint16_t) * d.np);
    d.mom = (float*)S->mom.ensure(sizeof(float) * d.np);
    d.vel = (float*)S->vel.ensure(sizeof(float) * d.np);
    S->grad.ensure(sizeof(float) * d.np);
    FH_HIP(hipMemcpyAsync(d.w, w.data(), sizeof(float) * d.np, hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipMemsetAsync(d.mom, 0, sizeof(float) * d.np, c.stream));
    FH_HIP(hipMemsetAsync(d.vel, 0, sizeof(float) * d.np, c.stream));
    const int npix = nz * ny * nx;
    std::vector<float> hf((size_t)std::max(1, nfields) * npix, 0.0f);
    for (size_t i = 0; i < (size_t)nfields * npix; ++i) hf[i] = (float)fields[i];
    d.fields = (const float*)S->fields.ensure(sizeof(float) * hf.size());
    FH_HIP(hipMemcpyAsync((void*)d.fields, hf.data(), sizeof(float) * hf.size(), hipMemcpyHostToDevice, c.stream));
    net_sync_bf16(c.stream, d);
    FH_HIP(hipStreamSynchronize(c.stream));
    return S;
}

void net_set_fields(Ctx& c, NetState& S, const double* fields) {
    const int nf = S.d.cin - NET_FIXED_CH;
    const long npix = S.d.npix();
    std::vector<float> hf((size_t)std::max(1, nf) * npix, 0.0f);
    for (size_t i = 0; i < (size_t)nf * npix; ++i) hf[i] = (float)fields[i];
    FH_HIP(hipMemcpyAsync((void*)S.d.fields, hf.data(), sizeof(float) * hf.size(), hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
}

void net_set_activations(NetState& S, int bf16) { S.d.bf16_act = bf16; }

void net_set_params(Ctx& c, NetState& S, const float* host) {
    FH_HIP(hipMemcpyAsync(S.d.w, host, sizeof(float) * S.d.np, hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipMemsetAsync(S.d.mom, 0, sizeof(float) * S.d.np, c.stream));
    FH_HIP(hipMemsetAsync(S.d.vel, 0, sizeof(float) * S.d.np, c.stream));
    S.d.t = 0;
    net_sync_bf16(c.stream, S.d);
    FH_HIP(hipStreamSynchronize(c.stream));
}

void net_get_params(Ctx& c, NetState& S, float* host) {
    FH_HIP(hipMemcpyAsync(host, S.d.w, sizeof(float) * S.d.np, hipMemcpyDeviceToHost, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
}

// activations for a batch of mt columns
static void ensure_acts(NetState& S, long npix, int mt) {
    S.x.ensure(sizeof(float) * npix * S.d.cin * mt);
    S.a1.ensure(sizeof(float) * npix * NET_HID * mt);
    S.a2.ensure(sizeof(float) * npix * NET_HID * mt);
    S.out.ensure(sizeof(float) * npix * 2 * mt);
    S.s1.ensure(sizeof(uint16_t) * 2 * npix * 16 * mt);
    S.s2.ensure(sizeof(uint16_t) * 2 * npix * 16 * mt);
}

static void upload_sys(Ctx& c, NetState& S, int nsys, const double* shifts, const int* sides) {
    FH_HIP(hipMemcpyAsync(S.shifts.ensure(sizeof(zd) * nsys), shifts, sizeof(zd) * nsys, hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipMemcpyAsync(S.sides.ensure(sizeof(int) * nsys), sides, sizeof(int) * nsys, hipMemcpyHostToDevice, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
}

// Activation workspace of the forward pass: about 300 bytes per (pixel, column)
// (FP32 inputs and hidden layers, their BF16 hi / lo splits, the output).  A
// pass covers at most NET_PASS_BYTES of it: the systems in groups, or one
// system in windows of its columns (a multiple of 16) when its m columns do
// not fit.
constexpr double NET_PASS_BYTES = 6e9;

template <typename T>
void net_apply(Ctx& c, NetState& S, int nsys, int m, const Cx<T>* V, const zd* shifts_dev, const int* sides_dev,
               Cx<T>* Out, bool unit_columns) {
    const long npix = (long)S.d.npix();
    const double per_col = (double)npix * (4.0 * (S.d.cin + 2 * NET_HID + 2) + 4.0 * 2 * 16);
    const int cap = std::max(16, (int)(NET_PASS_BYTES / per_col) / 16 * 16);
    const int mc = std::min(m, cap);                        // columns of a window
    const int gs = std::max(1, std::min(nsys, cap / std::max(1, mc)));   // systems of a group
    const long blk = npix * m;
    for (int s0 = 0; s0 < nsys; s0 += gs) {
        const int g = std::min(gs, nsys - s0);
        for (int c0 = 0; c0 < m; c0 += mc) {
            const int w = std::min(mc, m - c0);
            const int mt = g * w;
            ensure_acts(S, npix, mt);
            float* sc = nullptr;
            if (!unit_columns) {
                sc = (float*)S.scale.ensure(sizeof(float) * mt);
                net_inv_colnorm<T>(c.stream, S.d, w, g, V + s0 * blk, sc, m, c0);
            }
            net_encode<T>(c.stream, S.d, w, g, V + s0 * blk, sc, shifts_dev + s0, sides_dev + s0, (float*)S.x.p, m,
                          c0);
            net_forward(c.stream, S.d, mt, (const float*)S.x.p, (float*)S.a1.p, (float*)S.a2.p, (float*)S.out.p,
                        (uint16_t*)S.s1.p, (uint16_t*)S.s2.p, S.d.bf16_act != 0);
            net_decode<T>(c.stream, S.d, w, g, (const float*)S.out.p, sc, Out + s0 * blk, m, c0);
        }
    }
}
template void net_apply<double>(Ctx&, NetState&, int, int, const zd*, const zd*, const int*, zd*, bool);
template void net_apply<float>(Ctx&, NetState&, int, int, const cf*, const zd*, const int*, cf*, bool);

void net_forward_host(Ctx& c, NetState& S, int nsys, int m, const zd* X, const double* shifts, const int* sides,
                      zd* Out) {
    upload_sys(c, S, nsys, shifts, sides);
    net_apply<double>(c, S, nsys, m, X, (const zd*)S.shifts.p, (const int*)S.sides.p, Out, false);
    FH_HIP(hipStreamSynchronize(c.stream));
}

// Operator-weighted loss and its output gradient (o-space): with d = o - t
// per column, loss_c = ||M d||^2 / ||M t||^2 and dL/do = 2 M^H M d / (||M t||^2 mt),
// M the column's shifted operator (op shift z: right z - A, left z - A^H).
static double op_loss_grad(Ctx& c, NetState& S, const SparseState& sp, int nsys, int m, const double* shifts,
                           const int* sides, const float* out, const float* tgt, float* gout) {
    hipStream_t st = c.stream;
    const int n = sp.n;
    const long blk = (long)n * m, len = blk * nsys;
    const int mt = nsys * m;
    zd* D = (zd*)S.opD.ensure(sizeof(zd) * len);
    zd* T = (zd*)S.opT.ensure(sizeof(zd) * len);
    zd* MD = (zd*)S.opMD.ensure(sizeof(zd) * len);
    zd* MT = (zd*)S.opMT.ensure(sizeof(zd) * len);
    zd* G = (zd*)S.opG.ensure(sizeof(zd) * len);
    // op shifts and their conjugates (the adjoint's shifts)
    std::vector<zd> hs(2 * (size_t)nsys);
    for (int k = 0; k < nsys; ++k) {
        hs[k] = zd{shifts[2 * k], shifts[2 * k + 1]};
        hs[nsys + k] = zd{shifts[2 * k], -shifts[2 * k + 1]};
    }
    zd* dsh = (zd*)S.opsh.ensure(sizeof(zd) * 2 * nsys);
    FH_HIP(hipMemcpyAsync(dsh, hs.data(), sizeof(zd) * 2 * nsys, hipMemcpyHostToDevice, st));
    net_pack_diff(st, S.d, m, nsys, out, tgt, D, T);
    for (int k = 0; k < nsys; ++k) {
        const CsrDev& op = sides[k] ? sp.AT : sp.A;
        spmm<double>(st, op, sides[k] == 1, n, m, 1, dsh + k, 1.0, D + k * blk, nullptr, MD + k * blk);
        spmm<double>(st, op, sides[k] == 1, n, m, 1, dsh + k, 1.0, T + k * blk, nullptr, MT + k * blk);
    }
    double* nrm = (double*)S.opn.ensure(sizeof(double) * 2 * mt);
    colnorms<double>(st, n, m, nsys, MD, nrm, S.part);
    colnorms<double>(st, n, m, nsys, MT, nrm + mt, S.part);
    std::vector<double> h(2 * (size_t)mt), f(mt);
    FH_HIP(hipMemcpyAsync(h.data(), nrm, sizeof(double) * 2 * mt, hipMemcpyDeviceToHost, st));
    FH_HIP(hipStreamSynchronize(st));
    double loss = 0.0;
    for (int q = 0; q < mt; ++q) {
        const double den = h[mt + q] > 0 ? h[mt + q] * h[mt + q] : 1.0;
        loss += h[q] * h[q] / den;
        f[q] = 2.0 / (den * mt);
    }
    double* df = (double*)S.opf.ensure(sizeof(double) * mt);
    FH_HIP(hipMemcpyAsync(df, f.data(), sizeof(double) * mt, hipMemcpyHostToDevice, st));
    // G = M^H (M d): the adjoint of a right system is conj(z) - A^H, of a left one conj(z) - A
    for (int k = 0; k < nsys; ++k) {
        const CsrDev& adj = sides[k] ? sp.A : sp.AT;
        spmm<double>(st, adj, sides[k] == 0, n, m, 1, dsh + nsys + k, 1.0, MD + k * blk, nullptr, G + k * blk);
    }
    net_grad_encode(st, S.d, m, nsys, G, df, gout);
    FH_HIP(hipStreamSynchronize(st));
    return loss / mt;
}

// loss of the batch and the parameter gradient (left in S.grad); optionally an Adam step.
// sp == nullptr: plain error loss; else the operator-weighted loss of sp's operator.
double net_loss_grad(Ctx& c, NetState& S, const SparseState* sp, int nsys, int m, const zd* R, const zd* E,
                     const double* shifts, const int* sides, bool step, double lr) {
    upload_sys(c, S, nsys, shifts, sides);
    const long npix = (long)S.d.npix();
    const int mt = nsys * m;
    ensure_acts(S, npix, mt);
    float* sc = (float*)S.scale.ensure(sizeof(float) * mt);
    net_inv_colnorm<double>(c.stream, S.d, m, nsys, R, sc);     // inputs and targets scaled by 1/||r||
    net_encode<double>(c.stream, S.d, m, nsys, R, sc, (const zd*)S.shifts.p, (const int*)S.sides.p, (float*)S.x.p);
    float* tgt = (float*)S.tgt.ensure(sizeof(float) * npix * 2 * mt);
    net_target<double>(c.stream, S.d, m, nsys, E, sc, tgt);
    net_forward(c.stream, S.d, mt, (const float*)S.x.p, (float*)S.a1.p, (float*)S.a2.p, (float*)S.out.p,
                (uint16_t*)S.s1.p, (uint16_t*)S.s2.p);
    float* gout = (float*)S.gout.ensure(sizeof(float) * npix * 2 * mt);
    const double loss = sp ? op_loss_grad(c, S, *sp, nsys, m, shifts, sides, (const float*)S.out.p, tgt, gout)
                           : net_loss(c.stream, S.d, mt, (const float*)S.out.p, tgt, gout, S.lossbuf);
    float* g2 = (float*)S.g2.ensure(sizeof(float) * npix * NET_HID * mt);
    float* g1 = (float*)S.g1.ensure(sizeof(float) * npix * NET_HID * mt);
    net_backward(c.stream, S.d, mt, (const float*)S.x.p, (const float*)S.a1.p, (const float*)S.a2.p, gout, g2, g1,
                 (float*)S.grad.p, S.part, (uint16_t*)S.s1.p);
    if (step) net_adam(c.stream, S.d, (const float*)S.grad.p, (float)lr);
    FH_HIP(hipStreamSynchronize(c.stream));
    return loss;
}

void net_destroy(NetState* s) { delete s; }
int net_param_count(const NetState* s) { return s->d.np; }
int net_field_count(const NetState* s) { return s->d.cin - NET_FIXED_CH; }
int net_grid_size(const NetState* s) { return s->d.npix(); }
void net_get_grad(Ctx& c, NetState& S, float* host) {
    FH_HIP(hipMemcpyAsync(host, S.grad.p, sizeof(float) * S.d.np, hipMemcpyDeviceToHost, c.stream));
    FH_HIP(hipStreamSynchronize(c.stream));
}

}  // namespace fh
