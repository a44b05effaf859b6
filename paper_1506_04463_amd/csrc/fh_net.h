// Learned-preconditioner network state and launchers (k_net.hip, net.cpp).
#pragma once
#include <cstring>
#include <vector>

#include "fh_internal.h"

namespace fh {

constexpr int NET_HID = 16;       // hidden channels
constexpr int NET_MAX_CIN = 16;   // input channels of any layer
constexpr int NET_MAX_COUT = 16;
constexpr int NET_FIXED_CH = 5;   // Re r, Im r, Re z/alpha, Im z/alpha, side
constexpr int NET_WG_THREADS = NET_MAX_COUT * (NET_MAX_CIN + 1);   // 272

// device view of the network (pointers into NetState buffers)
struct NetDev {
    int nz = 1, ny = 0, nx = 0, cin = NET_FIXED_CH, np = 0, t = 0;
    int taps = 9;                // 9 (2D grid, nz = 1) or 27 (3D grid)
    double inv_alpha = 1.0;
    float oscale = 1.0f;         // output scale: e = ||r|| oscale (o_0 + i o_1)
    int bf16_act = 0;            // inference passes: 1 = BF16 activations, 0 = FP32 (two BF16 terms)
    int off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
    float* w = nullptr;          // FP32 master parameters
    uint16_t* wb = nullptr;      // BF16 copy used by the kernels
    float* mom = nullptr;        // Adam first moment
    float* vel = nullptr;        // Adam second moment
    const float* fields = nullptr;   // [nfields][npix]
    __host__ __device__ int npix() const { return nz * ny * nx; }
};

template <typename T>
void net_encode(hipStream_t st, const NetDev& N, int m, int nsys, const Cx<T>* V, const float* scale, const zd* shifts,
                const int* sides, float* x, int ld = 0, int c0 = 0);
template <typename T>
void net_decode(hipStream_t st, const NetDev& N, int m, int nsys, const float* o, const float* scale, Cx<T>* Out,
                int ld = 0, int c0 = 0);
template <typename T>
void net_target(hipStream_t st, const NetDev& N, int m, int nsys, const Cx<T>* E, const float* scale, float* t);
template <typename T>
void net_inv_colnorm(hipStream_t st, const NetDev& N, int m, int nsys, const Cx<T>* V, float* sc, int ld = 0,
                     int c0 = 0);
// s1, s2: split (BF16 hi / lo) workspaces of 2 x npix x 16 x mt entries each;
// bf16_act: single-term BF16 inputs of the MFMA layers, a1 not written
// (inference only: the backward pass needs the FP32 form)
void net_forward(hipStream_t st, const NetDev& N, int mt, const float* x, float* a1, float* a2, float* out,
                 uint16_t* s1, uint16_t* s2, bool bf16_act = false);
void net_backward(hipStream_t st, const NetDev& N, int mt, const float* x, const float* a1, const float* a2,
                  const float* gout, float* g2, float* g1, float* grad, DBuf& part, uint16_t* s1);
double net_loss(hipStream_t st, const NetDev& N, int mt, const float* out, const float* tgt, float* gout, DBuf& scratch);
void net_adam(hipStream_t st, NetDev& N, const float* grad, float lr);
void net_pack_diff(hipStream_t st, const NetDev& N, int m, int nsys, const float* o, const float* t, zd* D, zd* Tc);
void net_grad_encode(hipStream_t st, const NetDev& N, int m, int nsys, const zd* G, const double* f, float* gout);
void net_sync_bf16(hipStream_t st, NetDev& N);
uint16_t host_f32_to_bf16(float f);

struct NetState {
    NetDev d;
    DBuf w, wb, mom, vel, fields, grad;
    DBuf x, a1, a2, out, tgt, g1, g2, gout, scale, shifts, sides, part, lossbuf;
    DBuf s1, s2;   // BF16 hi / lo splits of the MFMA layers' inputs
    DBuf opD, opT, opMD, opMT, opG, opsh, opn, opf;   // operator-weighted loss
};

// apply the network to a batch of blocks ([nsys][n][m], unit or arbitrary
// column norms): Out = ||v|| * net(v / ||v||, shift, side)
template <typename T>
void net_apply(Ctx& c, NetState& S, int nsys, int m, const Cx<T>* V, const zd* shifts_dev, const int* sides_dev,
               Cx<T>* Out, bool unit_columns);

}  // namespace fh
