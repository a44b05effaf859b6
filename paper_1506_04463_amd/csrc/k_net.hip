// Learned preconditioner: a 3-layer 3x3 convolutional network on the solution
// grid (Cin -> H -> H -> 2 channels, zero padding, ReLU between layers), with
// weights stored in BF16 and FP32 accumulation; forward, backward (data and
// weights) and Adam kernels used to train it on (residual, error) pairs and
// to apply it as a flexible preconditioner inside FGMRES.
//
// Activation layout: [pixel][channel][column] (FP32), pixel = (z * ny + y) * nx + x;
// the columns of a batch are contiguous, so every access is coalesced across
// the batch.  Weight layout: [Cout][Cin][TAPS], TAPS = 9 on a 2D grid (tap =
// (dy+1)*3 + (dx+1)) or 27 on a 3D grid (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)).
#include "fh_net.h"

namespace fh {

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    // round to nearest even
    uint32_t u;
#ifdef __HIP_DEVICE_COMPILE__
    u = __float_as_uint(f);
#else
    std::memcpy(&u, &f, 4);
#endif
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

// offsets of a tap along z, y, x
template <int TAPS>
__device__ __forceinline__ void tap_off(int tap, int& dz, int& dy, int& dx) {
    dz = TAPS == 27 ? tap / 9 - 1 : 0;
    dy = (tap % 9) / 3 - 1;
    dx = tap % 3 - 1;
}

// ---------------------------------------------------------------------------
// input encoding: x[p][ch][col], col = s*m + c:
//   ch 0, 1: Re/Im of V[s][p][c] * scale[col]; ch 2, 3: Re/Im of shift_s / alpha;
//   ch 4: side_s; ch 5..: fields[f][p]
// ---------------------------------------------------------------------------
// V rows of ld entries (ld >= m): column c of the window is entry c0 + c
template <typename T>
__global__ void k_net_encode(int npix, int m, int nsys, int cin, const Cx<T>* __restrict__ V, int ld, int c0,
                             const float* __restrict__ scale, const zd* __restrict__ shifts, const int* __restrict__ sides,
                             double inv_alpha, const float* __restrict__ fields, float* __restrict__ x) {
    const int mt = nsys * m;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)npix * mt) return;
    const int p = e / mt, col = e % mt;
    const int s = col / m, c = col % m;
    const Cx<T> v = V[(long)s * npix * ld + (long)p * ld + c0 + c];
    const float sc = scale ? scale[col] : 1.0f;
    float* xp = x + (long)p * cin * mt + col;
    xp[0] = (float)v.re * sc;
    xp[(long)mt] = (float)v.im * sc;
    const zd z = shifts[s];
    xp[2L * mt] = (float)(z.re * inv_alpha);
    xp[3L * mt] = (float)(z.im * inv_alpha);
    xp[4L * mt] = (float)sides[s];
    for (int f = 0; f < cin - NET_FIXED_CH; ++f) xp[(long)(NET_FIXED_CH + f) * mt] = fields[(long)f * npix + p];
}

// Out[s][p][c] = oscale (o[p][0][col] + i o[p][1][col]) / scale[col]  (scale = 1/||r|| of the input)
template <typename T>
__global__ void k_net_decode(int npix, int m, int nsys, float oscale, const float* __restrict__ o,
                             const float* __restrict__ scale, Cx<T>* __restrict__ Out, int ld, int c0) {
    const int mt = nsys * m;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)npix * mt) return;
    const int p = e / mt, col = e % mt;
    const int s = col / m, c = col % m;
    const float sc = scale ? scale[col] : 1.0f;
    const float inv = sc > 0.0f ? oscale / sc : 0.0f;
    const float* op = o + (long)p * 2 * mt + col;
    Out[(long)s * npix * ld + (long)p * ld + c0 + c] = Cx<T>{T(op[0] * inv), T(op[mt] * inv)};
}

// ---------------------------------------------------------------------------
// forward 3x3 convolution: one thread per (pixel, column), all COUT outputs
// ---------------------------------------------------------------------------
template <int COUT, int TAPS>
__global__ __launch_bounds__(256) void k_conv_fwd(int nz, int ny, int nx, int mt, int cin, const float* __restrict__ x,
                                                  const uint16_t* __restrict__ w, const uint16_t* __restrict__ b,
                                                  int relu, float* __restrict__ y) {
    __shared__ float ws[COUT * NET_MAX_CIN * TAPS];
    __shared__ float bs[COUT];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (int i = tid; i < COUT * cin * TAPS; i += blockDim.x * blockDim.y) ws[i] = bf16_to_f32(w[i]);
    if (tid < COUT) bs[tid] = bf16_to_f32(b[tid]);
    __syncthreads();
    const int col = blockIdx.y * blockDim.x + threadIdx.x;
    const int p = blockIdx.x * blockDim.y + threadIdx.y;
    if (col >= mt || p >= nz * ny * nx) return;
    const int px = p % nx, py = (p / nx) % ny, pz = p / (nx * ny);
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; ++o) acc[o] = bs[o];
    for (int tap = 0; tap < TAPS; ++tap) {
        int dz, dy, dx;
        tap_off<TAPS>(tap, dz, dy, dx);
        const int qz = pz + dz, qy = py + dy, qx = px + dx;
        if (qz < 0 || qz >= nz || qy < 0 || qy >= ny || qx < 0 || qx >= nx) continue;
        const float* xq = x + (long)((qz * ny + qy) * nx + qx) * cin * mt + col;
        for (int ci = 0; ci < cin; ++ci) {
            const float v = xq[(long)ci * mt];
#pragma unroll
            for (int o = 0; o < COUT; ++o) acc[o] = fmaf(ws[(o * cin + ci) * TAPS + tap], v, acc[o]);
        }
    }
    float* yp = y + (long)p * COUT * mt + col;
#pragma unroll
    for (int o = 0; o < COUT; ++o) yp[(long)o * mt] = relu ? fmaxf(acc[o], 0.0f) : acc[o];
}

// ---------------------------------------------------------------------------
// 16-channel convolutions on MFMA (v_mfma_f32_16x16x16_bf16).  Per pixel the
// [16 channels][16 columns] output block is a sum over taps of a 16 x 16 BF16
// weight block times the neighbour's [16 channels][16 columns] input block.
// Lane l of a wave supplies A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16]
// (j = 0..3) and receives D[4 (l / 16) + v][l % 16] (v = 0..3).  The weights are
// BF16 already; each FP32 input enters as two BF16 terms, x = hi + lo to
// 2^-17 relative, so that the result keeps FP32-level accuracy; the
// accumulation is FP32.  The inputs are split once, into "split" arrays of
// layout [pixel][channel / 4][column][4] (hi and lo arrays of 16 channels), so
// that a lane's B operand is one 8-byte load and no tap repeats the split.
// A wave computes 16 columns of MFMA_PPW consecutive pixels with all taps'
// weight blocks held in registers.
// ---------------------------------------------------------------------------
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int MFMA_PPW = 8;    // pixels per wave

__device__ __forceinline__ void split_bf16(float v, short& hi, short& lo) {
    const uint16_t h = f32_to_bf16(v);
    hi = (short)h;
    lo = (short)f32_to_bf16(v - bf16_to_f32(h));
}

// split arrays of x[p][ci][col] (cin <= 16 channels, zero padded to 16):
// hi/lo[((p * 4 + cq) * mt + col) * 4 + j] for ci = 4 cq + j (lo may be null:
// BF16 activations, the hi term only)
__global__ void k_split16(long npix, int mt, int cin, const float* __restrict__ x, bf16x4_t* __restrict__ hi,
                          bf16x4_t* __restrict__ lo) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;   // (p, cq, col)
    if (e >= npix * 4 * mt) return;
    const int col = (int)(e % mt);
    const long pq = e / mt;
    const int cq = (int)(pq % 4);
    const long p = pq / 4;
    bf16x4_t h, l;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int ci = 4 * cq + j;
        const float v = ci < cin ? x[(p * cin + ci) * mt + col] : 0.0f;
        short a, b;
        split_bf16(v, a, b);
        h[j] = a;
        l[j] = b;
    }
    hi[e] = h;
    if (lo) lo[e] = l;
}

// One kernel for both directions.  Forward: y[p][co][col] = act(b[co] +
// sum_{tap, ci} w[co][ci][tap] x[p + d(tap)][ci][col]), 16 outputs, cin <= 16,
// and the split of y when yhi != null.  Backward (BWD): dx[p][ci][col] =
// mask(p, ci) sum_{co, tap} w[co][ci][tap] dy[p - d(tap)][co][col] (16 and 16
// channels; mask: a_prev > 0, or none).  A wave computes MFMA_PPW consecutive
// pixels of one grid row (x fastest) for 16 columns; for each (dz, dy) plane
// it loads the MFMA_PPW + 2 input blocks of the row window once and uses each
// for up to three taps and three output pixels (a neighbour outside the grid
// contributes a zero operand).
template <int TAPS, bool BWD, int NTERM = 2>
__global__ __launch_bounds__(256) void k_conv16_mfma(int nz, int ny, int nx, int mt, int cin,
                                                     const bf16x4_t* __restrict__ xhi, const bf16x4_t* __restrict__ xlo,
                                                     const uint16_t* __restrict__ w, const uint16_t* __restrict__ b,
                                                     int relu, const float* __restrict__ mask, float* __restrict__ y,
                                                     bf16x4_t* __restrict__ yhi, bf16x4_t* __restrict__ ylo) {
    constexpr int PP = MFMA_PPW, WIN = MFMA_PPW + 2;
    constexpr int NPL = TAPS == 27 ? 9 : 3;          // (dz, dy) planes
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i16 = lane & 15, kq = lane >> 4;
    const int col = blockIdx.y * 16 + i16;
    const bool colok = col < mt;
    const int segs = (nx + PP - 1) / PP;
    const long task = (long)blockIdx.x * 4 + wave;   // (z, y, segment)
    if (task >= (long)nz * ny * segs) return;        // uniform over the wave; no barrier below
    const int seg = (int)(task % segs);
    const int py = (int)((task / segs) % ny), pz = (int)(task / ((long)segs * ny));
    const int px0 = seg * PP;
    bf16x4_t wa[TAPS];
#pragma unroll
    for (int tap = 0; tap < TAPS; ++tap)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (!BWD) {
                const int ci = 4 * kq + j;
                wa[tap][j] = ci < cin ? (short)w[(i16 * cin + ci) * TAPS + tap] : (short)0;
            } else {
                wa[tap][j] = (short)w[((4 * kq + j) * 16 + i16) * TAPS + tap];   // A[ci][co]
            }
        }
    const bf16x4_t zero4 = {0, 0, 0, 0};
    f32x4_t acc[PP];
#pragma unroll
    for (int i = 0; i < PP; ++i) acc[i] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
    const int sg = BWD ? -1 : 1;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl) {
        const int dz = TAPS == 27 ? pl / 3 - 1 : 0, dy = pl % 3 - 1;
        const int qz = pz + sg * dz, qy = py + sg * dy;
        const bool plane = qz >= 0 && qz < nz && qy >= 0 && qy < ny && colok;
        const long rowbase = plane ? (long)(qz * ny + qy) * nx : 0;
        bf16x4_t hi[WIN], lo[WIN];
#pragma unroll
        for (int u = 0; u < WIN; ++u) {
            const int qx = px0 - 1 + u;
            const bool in = plane && qx >= 0 && qx < nx;
            const long e = ((in ? rowbase + qx : 0L) * 4 + kq) * mt + (colok ? col : 0);
            const bf16x4_t hl = xhi[e];
            hi[u] = in ? hl : zero4;
            if (NTERM == 2) {
                const bf16x4_t ll = xlo[e];
                lo[u] = in ? ll : zero4;
            }
        }
#pragma unroll
        for (int i = 0; i < PP; ++i)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const int tap = (TAPS == 27 ? (dz + 1) * 9 : 0) + (dy + 1) * 3 + (dx + 1);
                const int u = i + 1 + sg * dx;
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[tap], hi[u], acc[i], 0, 0, 0);
                if (NTERM == 2) acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(wa[tap], lo[u], acc[i], 0, 0, 0);
            }
    }
    if (!colok) return;
    float bias[4];
    if (!BWD) {
#pragma unroll
        for (int v = 0; v < 4; ++v) bias[v] = bf16_to_f32(b[4 * kq + v]);
    }
#pragma unroll
    for (int i = 0; i < PP; ++i) {
        const int px = px0 + i;
        if (px >= nx) break;
        const long p = (long)(pz * ny + py) * nx + px;
        float* yp = y + p * 16 * mt + col;
        if (!BWD) {
            bf16x4_t h, l;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float o = acc[i][v] + bias[v];
                if (relu) o = fmaxf(o, 0.0f);
                if (y) yp[(long)(4 * kq + v) * mt] = o;
                short a, c;
                split_bf16(o, a, c);
                h[v] = a;
                l[v] = c;
            }
            if (yhi) {
                const long e = (p * 4 + kq) * mt + col;
                yhi[e] = h;
                if (ylo) ylo[e] = l;
            }
        } else {
            const float* mp = mask ? mask + p * 16 * mt + col : nullptr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long o = (long)(4 * kq + v) * mt;
                yp[o] = (mp && !(mp[o] > 0.0f)) ? 0.0f : acc[i][v];
            }
        }
    }
}

static dim3 mfma_grid(const NetDev& N, int mt) {
    const long tasks = (long)N.nz * N.ny * ceil_div(N.nx, MFMA_PPW);
    return dim3((unsigned)ceil_div(tasks, 4), ceil_div(mt, 16));
}

// ---------------------------------------------------------------------------
// backward (data): dx[p][ci][col] = mask(p, ci) * sum_{o,tap} w[o][ci][tap] dy[p - d(tap)][o][col]
// mask: a_prev[p][ci][col] > 0 (ReLU of the layer input), or none
// ---------------------------------------------------------------------------
template <int CIN, int TAPS>
__global__ __launch_bounds__(256) void k_conv_bwd_data(int nz, int ny, int nx, int mt, int cout,
                                                       const float* __restrict__ dy, const uint16_t* __restrict__ w,
                                                       const float* __restrict__ mask, float* __restrict__ dx) {
    __shared__ float ws[NET_MAX_COUT * CIN * TAPS];
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (int i = tid; i < cout * CIN * TAPS; i += blockDim.x * blockDim.y) ws[i] = bf16_to_f32(w[i]);
    __syncthreads();
    const int col = blockIdx.y * blockDim.x + threadIdx.x;
    const int p = blockIdx.x * blockDim.y + threadIdx.y;
    if (col >= mt || p >= nz * ny * nx) return;
    const int px = p % nx, py = (p / nx) % ny, pz = p / (nx * ny);
    float acc[CIN];
#pragma unroll
    for (int c = 0; c < CIN; ++c) acc[c] = 0.0f;
    for (int tap = 0; tap < TAPS; ++tap) {
        // output pixel q = p - d feeds input p through tap
        int ddz, ddy, ddx;
        tap_off<TAPS>(tap, ddz, ddy, ddx);
        const int qz = pz - ddz, qy = py - ddy, qx = px - ddx;
        if (qz < 0 || qz >= nz || qy < 0 || qy >= ny || qx < 0 || qx >= nx) continue;
        const float* dq = dy + (long)((qz * ny + qy) * nx + qx) * cout * mt + col;
        for (int o = 0; o < cout; ++o) {
            const float g = dq[(long)o * mt];
#pragma unroll
            for (int c = 0; c < CIN; ++c) acc[c] = fmaf(ws[(o * CIN + c) * TAPS + tap], g, acc[c]);
        }
    }
    float* dxp = dx + (long)p * CIN * mt + col;
    const float* mp = mask ? mask + (long)p * CIN * mt + col : nullptr;
#pragma unroll
    for (int c = 0; c < CIN; ++c) dxp[(long)c * mt] = (mp && !(mp[(long)c * mt] > 0.0f)) ? 0.0f : acc[c];
}

// ---------------------------------------------------------------------------
// backward (weights): thread (o, ci) accumulates, for the 9 taps,
// sum over its pixel slice and all columns of dy[p][o][col] * x[p + d][ci][col];
// the slice's rows are staged through LDS in 64-column chunks.  Bias gradient
// by the threads with ci == cin (extra row).  Partials [slice][o][cin+1][9].
// ---------------------------------------------------------------------------
constexpr int WG_SLICE = 8;     // pixels per workgroup

template <int TAPS>
__global__ __launch_bounds__(320) void k_conv_bwd_weight(int nz, int ny, int nx, int mt, int cin, int cout,
                                                         const float* __restrict__ x, const float* __restrict__ dy,
                                                         float* __restrict__ part) {
    constexpr int WGC = TAPS == 27 ? 16 : 32;    // columns per LDS chunk
    __shared__ float dys[NET_MAX_COUT][WGC];
    __shared__ float xs[TAPS][NET_MAX_CIN][WGC];
    const int tid = threadIdx.x;
    const int o = tid / (NET_MAX_CIN + 1), ci = tid % (NET_MAX_CIN + 1);
    const bool active = (tid < NET_WG_THREADS) && (o < cout) && (ci <= cin);
    const int nth = blockDim.x;
    float acc[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) acc[t] = 0.0f;
    const int npix = nz * ny * nx;
    const int p0 = blockIdx.x * WG_SLICE;
    for (int p = p0; p < min(npix, p0 + WG_SLICE); ++p) {
        const int px = p % nx, py = (p / nx) % ny, pz = p / (nx * ny);
        for (int c0 = 0; c0 < mt; c0 += WGC) {
            const int cw = min(WGC, mt - c0);
            for (int e = tid; e < cout * WGC; e += nth) {
                const int oo = e / WGC, cc = e % WGC;
                dys[oo][cc] = (cc < cw) ? dy[(long)p * cout * mt + (long)oo * mt + c0 + cc] : 0.0f;
            }
            for (int e = tid; e < TAPS * cin * WGC; e += nth) {
                const int tap = e / (cin * WGC), rem = e % (cin * WGC);
                const int cc2 = rem / WGC, cc = rem % WGC;
                int dz, dyy, dx;
                tap_off<TAPS>(tap, dz, dyy, dx);
                const int qz = pz + dz, qy = py + dyy, qx = px + dx;
                float v = 0.0f;
                if (cc < cw && qz >= 0 && qz < nz && qy >= 0 && qy < ny && qx >= 0 && qx < nx)
                    v = x[(long)((qz * ny + qy) * nx + qx) * cin * mt + (long)cc2 * mt + c0 + cc];
                xs[tap][cc2][cc] = v;
            }
            __syncthreads();
            if (active) {
                for (int cc = 0; cc < cw; ++cc) {
                    const float g = dys[o][cc];
                    if (ci < cin) {
#pragma unroll
                        for (int t = 0; t < TAPS; ++t) acc[t] = fmaf(g, xs[t][ci][cc], acc[t]);
                    } else {
                        acc[0] += g;       // bias
                    }
                }
            }
            __syncthreads();
        }
    }
    if (active) {
        float* pp = part + ((long)blockIdx.x * NET_MAX_COUT * (NET_MAX_CIN + 1) + (long)o * (NET_MAX_CIN + 1) + ci) * TAPS;
#pragma unroll
        for (int t = 0; t < TAPS; ++t) pp[t] = acc[t];
    }
}

// sum the partials of the slices into the gradient (weights [o][ci][TAPS], then bias [o])
__global__ void k_wgrad_reduce(int nslice, int cin, int cout, int taps, const float* __restrict__ part,
                               float* __restrict__ gw, float* __restrict__ gb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int per = (NET_MAX_CIN + 1) * taps;
    if (e >= cout * (cin + 1) * taps) return;
    const int o = e / ((cin + 1) * taps), rem = e % ((cin + 1) * taps);
    const int ci = rem / taps, t = rem % taps;
    double s = 0.0;
    for (int k = 0; k < nslice; ++k) s += part[(long)k * NET_MAX_COUT * per + (long)o * per + ci * taps + t];
    if (ci < cin) gw[(o * cin + ci) * taps + t] = (float)s;
    else if (t == 0) gb[o] = (float)s;
}

// ---------------------------------------------------------------------------
// loss: per column sum (out - tgt)^2 / sum tgt^2, gradient 2 (out - tgt) / tn / mt
// ---------------------------------------------------------------------------
__global__ void k_loss_cols(int npix, int mt, const float* __restrict__ out, const float* __restrict__ tgt,
                            double* __restrict__ num, double* __restrict__ den) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= mt) return;
    double a = 0.0, b = 0.0;
    for (int p = 0; p < npix; ++p)
        for (int ch = 0; ch < 2; ++ch) {
            const float o = out[(long)p * 2 * mt + (long)ch * mt + col];
            const float t = tgt[(long)p * 2 * mt + (long)ch * mt + col];
            a += (double)(o - t) * (o - t);
            b += (double)t * t;
        }
    num[col] = a;
    den[col] = b > 0 ? b : 1.0;
}
__global__ void k_loss_grad(int npix, int mt, const float* __restrict__ out, const float* __restrict__ tgt,
                            const double* __restrict__ den, float* __restrict__ g) {
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)npix * 2 * mt) return;
    const int col = e % mt;
    g[e] = (float)(2.0 * ((double)out[e] - tgt[e]) / den[col] / mt);
}

// target encoding: t[p][0/1][col] = Re/Im(E[s][p][c]) * scale[col] / oscale
template <typename T>
__global__ void k_net_target(int npix, int m, int nsys, float inv_oscale, const Cx<T>* __restrict__ E,
                             const float* __restrict__ scale, float* __restrict__ t) {
    const int mt = nsys * m;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)npix * mt) return;
    const int p = e / mt, col = e % mt;
    const int s = col / m, c = col % m;
    const Cx<T> v = E[(long)s * npix * m + (long)p * m + c];
    const float sc = (scale ? scale[col] : 1.0f) * inv_oscale;
    t[(long)p * 2 * mt + col] = (float)v.re * sc;
    t[(long)p * 2 * mt + mt + col] = (float)v.im * sc;
}

// operator-weighted loss: D[s][p][c] = (o - t)[p][.][col], Tc[s][p][c] = t[p][.][col] as complex FP64
__global__ void k_net_pack_diff(int npix, int m, int nsys, const float* __restrict__ o, const float* __restrict__ t,
                                zd* __restrict__ D, zd* __restrict__ Tc) {
    const int mt = nsys * m;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)npix * mt) return;
    const int p = e / mt, col = e % mt;
    const int s = col / m, c = col % m;
    const long i2 = (long)p * 2 * mt + col;
    const long q = (long)s * npix * m + (long)p * m + c;
    D[q] = zd{(double)o[i2] - t[i2], (double)o[i2 + mt] - t[i2 + mt]};
    Tc[q] = zd{(double)t[i2], (double)t[i2 + mt]};
}

// gout[p][0/1][col] = f[col] * Re/Im G[s][p][c]
__global__ void k_net_grad_encode(int npix, int m, int nsys, const zd* __restrict__ G, const double* __restrict__ f,
                                  float* __restrict__ gout) {
    const int mt = nsys * m;
    long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)npix * mt) return;
    const int p = e / mt, col = e % mt;
    const int s = col / m, c = col % m;
    const zd g = G[(long)s * npix * m + (long)p * m + c];
    gout[(long)p * 2 * mt + col] = (float)(f[col] * g.re);
    gout[(long)p * 2 * mt + mt + col] = (float)(f[col] * g.im);
}

// Adam on the FP32 master parameters, then the BF16 copy
__global__ void k_adam(int np, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ mo,
                       float* __restrict__ ve, uint16_t* __restrict__ wb, float lr, float b1, float b2, float eps, int t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float m1 = b1 * mo[i] + (1.0f - b1) * gi;
    const float v1 = b2 * ve[i] + (1.0f - b2) * gi * gi;
    mo[i] = m1;
    ve[i] = v1;
    const float mh = m1 / (1.0f - powf(b1, (float)t));
    const float vh = v1 / (1.0f - powf(b2, (float)t));
    const float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
    w[i] = wi;
    wb[i] = f32_to_bf16(wi);
}
__global__ void k_to_bf16(int np, const float* __restrict__ w, uint16_t* __restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) wb[i] = f32_to_bf16(w[i]);
}

// per-column 1/||V col|| (0 for a zero column)
template <typename T>
__global__ void k_inv_colnorm(int npix, int m, int nsys, const Cx<T>* __restrict__ V, int ld, int c0,
                              float* __restrict__ sc) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    const int mt = nsys * m;
    if (col >= mt) return;
    const int s = col / m, c = col % m;
    double a = 0.0;
    for (int p = 0; p < npix; ++p) {
        const Cx<T> v = V[(long)s * npix * ld + (long)p * ld + c0 + c];
        a += (double)v.re * v.re + (double)v.im * v.im;
    }
    sc[col] = a > 0 ? (float)(1.0 / sqrt(a)) : 0.0f;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// pixel blocks along x (up to 2^31), column blocks along y
static dim3 conv_grid(int npix, int mt) { return dim3(ceil_div(npix, 4), ceil_div(mt, 64)); }

template <typename T>
void net_encode(hipStream_t st, const NetDev& N, int m, int nsys, const Cx<T>* V, const float* scale, const zd* shifts,
                const int* sides, float* x, int ld, int c0) {
    const long tot = (long)N.npix() * m * nsys;
    k_net_encode<T><<<ceil_div(tot, 256), 256, 0, st>>>(N.npix(), m, nsys, N.cin, V, ld > 0 ? ld : m, c0, scale,
                                                         shifts, sides, N.inv_alpha, N.fields, x);
    FH_LAUNCH_CHECK();
}
template <typename T>
void net_decode(hipStream_t st, const NetDev& N, int m, int nsys, const float* o, const float* scale, Cx<T>* Out,
                int ld, int c0) {
    const long tot = (long)N.npix() * m * nsys;
    k_net_decode<T><<<ceil_div(tot, 256), 256, 0, st>>>(N.npix(), m, nsys, N.oscale, o, scale, Out, ld > 0 ? ld : m,
                                                         c0);
    FH_LAUNCH_CHECK();
}
template <typename T>
void net_target(hipStream_t st, const NetDev& N, int m, int nsys, const Cx<T>* E, const float* scale, float* t) {
    const long tot = (long)N.npix() * m * nsys;
    k_net_target<T><<<ceil_div(tot, 256), 256, 0, st>>>(N.npix(), m, nsys, 1.0f / N.oscale, E, scale, t);
    FH_LAUNCH_CHECK();
}
template <typename T>
void net_inv_colnorm(hipStream_t st, const NetDev& N, int m, int nsys, const Cx<T>* V, float* sc, int ld, int c0) {
    k_inv_colnorm<T><<<ceil_div(m * nsys, 64), 64, 0, st>>>(N.npix(), m, nsys, V, ld > 0 ? ld : m, c0, sc);
    FH_LAUNCH_CHECK();
}
template void net_encode<double>(hipStream_t, const NetDev&, int, int, const zd*, const float*, const zd*, const int*, float*, int, int);
template void net_encode<float>(hipStream_t, const NetDev&, int, int, const cf*, const float*, const zd*, const int*, float*, int, int);
template void net_decode<double>(hipStream_t, const NetDev&, int, int, const float*, const float*, zd*, int, int);
template void net_decode<float>(hipStream_t, const NetDev&, int, int, const float*, const float*, cf*, int, int);
template void net_target<double>(hipStream_t, const NetDev&, int, int, const zd*, const float*, float*);
template void net_inv_colnorm<double>(hipStream_t, const NetDev&, int, int, const zd*, float*, int, int);
template void net_inv_colnorm<float>(hipStream_t, const NetDev&, int, int, const cf*, float*, int, int);

template <int TAPS>
static void forward_t(hipStream_t st, const NetDev& N, int mt, const float* x, float* a1, float* a2, float* out,
                      uint16_t* s1, uint16_t* s2, bool bf16_act) {
    const int npix = N.npix();
    dim3 blk(64, 4), g = conv_grid(npix, mt), gm = mfma_grid(N, mt);
    static_assert(NET_HID == 16 && NET_MAX_CIN <= 16, "the MFMA convolutions are 16-channel blocks");
    const long half = (long)npix * 16 * mt;      // bf16 entries of one split array
    bf16x4_t* x_hi = (bf16x4_t*)s1;
    bf16x4_t* x_lo = (bf16x4_t*)(s1 + half);
    bf16x4_t* a_hi = (bf16x4_t*)s2;
    bf16x4_t* a_lo = (bf16x4_t*)(s2 + half);
    if (bf16_act) {
        // inference with BF16 activations: the inputs of the two MFMA layers
        // are single BF16 terms (half the operand loads and MFMAs), the first
        // layer's FP32 output (needed only by the backward pass) is not stored
        k_split16<<<ceil_div((size_t)npix * 4 * mt, 256), 256, 0, st>>>(npix, mt, N.cin, x, x_hi, nullptr);
        FH_LAUNCH_CHECK();
        k_conv16_mfma<TAPS, false, 1><<<gm, 256, 0, st>>>(N.nz, N.ny, N.nx, mt, N.cin, x_hi, nullptr,
                                                          N.wb + N.off_w1, N.wb + N.off_b1, 1, nullptr, nullptr,
                                                          a_hi, nullptr);
        FH_LAUNCH_CHECK();
        k_conv16_mfma<TAPS, false, 1><<<gm, 256, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, a_hi, nullptr,
                                                          N.wb + N.off_w2, N.wb + N.off_b2, 1, nullptr, a2, nullptr,
                                                          nullptr);
        FH_LAUNCH_CHECK();
        k_conv_fwd<2, TAPS><<<g, blk, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, a2, N.wb + N.off_w3, N.wb + N.off_b3, 0,
                                               out);
        FH_LAUNCH_CHECK();
        return;
    }
    k_split16<<<ceil_div((size_t)npix * 4 * mt, 256), 256, 0, st>>>(npix, mt, N.cin, x, x_hi, x_lo);
    FH_LAUNCH_CHECK();
    k_conv16_mfma<TAPS, false><<<gm, 256, 0, st>>>(N.nz, N.ny, N.nx, mt, N.cin, x_hi, x_lo, N.wb + N.off_w1,
                                                   N.wb + N.off_b1, 1, nullptr, a1, a_hi, a_lo);
    FH_LAUNCH_CHECK();
    k_conv16_mfma<TAPS, false><<<gm, 256, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, a_hi, a_lo, N.wb + N.off_w2,
                                                   N.wb + N.off_b2, 1, nullptr, a2, nullptr, nullptr);
    FH_LAUNCH_CHECK();
    k_conv_fwd<2, TAPS><<<g, blk, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, a2, N.wb + N.off_w3, N.wb + N.off_b3, 0, out);
    FH_LAUNCH_CHECK();
}

void net_forward(hipStream_t st, const NetDev& N, int mt, const float* x, float* a1, float* a2, float* out,
                 uint16_t* s1, uint16_t* s2, bool bf16_act) {
    const int npix = N.npix();
    hipEvent_t ev = prof_begin(st);
    if (N.taps == 27) forward_t<27>(st, N, mt, x, a1, a2, out, s1, s2, bf16_act);
    else forward_t<9>(st, N, mt, x, a1, a2, out, s1, s2, bf16_act);
    const double macs = (double)N.taps * (N.cin * NET_HID + NET_HID * NET_HID + NET_HID * 2) * npix * mt;
    prof_end(st, ev, "net_forward", 4.0 * npix * mt * (N.cin + 2 * NET_HID + 2) * 2, 2 * macs);
}

template <int TAPS>
static void backward_t(hipStream_t st, const NetDev& N, int mt, const float* x, const float* a1, const float* a2,
                       const float* gout, float* g2, float* g1, float* grad, float* P, int nslice, uint16_t* s1) {
    dim3 blk(64, 4), g = conv_grid(N.npix(), mt);
    const int T = TAPS;
    // layer 3: weights, then data through ReLU(a2)
    k_conv_bwd_weight<TAPS><<<nslice, 320, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, 2, a2, gout, P);
    FH_LAUNCH_CHECK();
    k_wgrad_reduce<<<ceil_div(2 * (NET_HID + 1) * T, 128), 128, 0, st>>>(nslice, NET_HID, 2, T, P, grad + N.off_w3,
                                                                           grad + N.off_b3);
    FH_LAUNCH_CHECK();
    k_conv_bwd_data<NET_HID, TAPS><<<g, blk, 0, st>>>(N.nz, N.ny, N.nx, mt, 2, gout, N.wb + N.off_w3, a2, g2);
    FH_LAUNCH_CHECK();
    // layer 2
    k_conv_bwd_weight<TAPS><<<nslice, 320, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, NET_HID, a1, g2, P);
    FH_LAUNCH_CHECK();
    k_wgrad_reduce<<<ceil_div(NET_HID * (NET_HID + 1) * T, 128), 128, 0, st>>>(nslice, NET_HID, NET_HID, T, P,
                                                                                 grad + N.off_w2, grad + N.off_b2);
    FH_LAUNCH_CHECK();
    {
        const long half = (long)N.npix() * 16 * mt;
        bf16x4_t* g_hi = (bf16x4_t*)s1;
        bf16x4_t* g_lo = (bf16x4_t*)(s1 + half);
        k_split16<<<ceil_div((size_t)N.npix() * 4 * mt, 256), 256, 0, st>>>(N.npix(), mt, NET_HID, g2, g_hi, g_lo);
        FH_LAUNCH_CHECK();
        k_conv16_mfma<TAPS, true><<<mfma_grid(N, mt), 256, 0, st>>>(N.nz, N.ny, N.nx, mt, NET_HID, g_hi, g_lo,
                                                                     N.wb + N.off_w2, nullptr, 0, a1, g1, nullptr,
                                                                     nullptr);
    }
    FH_LAUNCH_CHECK();
    // layer 1 (weights only)
    k_conv_bwd_weight<TAPS><<<nslice, 320, 0, st>>>(N.nz, N.ny, N.nx, mt, N.cin, NET_HID, x, g1, P);
    FH_LAUNCH_CHECK();
    k_wgrad_reduce<<<ceil_div(NET_HID * (N.cin + 1) * T, 128), 128, 0, st>>>(nslice, N.cin, NET_HID, T, P,
                                                                               grad + N.off_w1, grad + N.off_b1);
    FH_LAUNCH_CHECK();
}

void net_backward(hipStream_t st, const NetDev& N, int mt, const float* x, const float* a1, const float* a2,
                  const float* gout, float* g2, float* g1, float* grad, DBuf& part, uint16_t* s1) {
    const int nslice = ceil_div(N.npix(), WG_SLICE);
    float* P = (float*)part.ensure(sizeof(float) * (size_t)nslice * NET_MAX_COUT * (NET_MAX_CIN + 1) * N.taps);
    hipEvent_t ev = prof_begin(st);
    if (N.taps == 27) backward_t<27>(st, N, mt, x, a1, a2, gout, g2, g1, grad, P, nslice, s1);
    else backward_t<9>(st, N, mt, x, a1, a2, gout, g2, g1, grad, P, nslice, s1);
    const double macs = (double)N.taps * (N.cin * NET_HID + NET_HID * NET_HID + NET_HID * 2) * N.npix() * mt;
    prof_end(st, ev, "net_backward", 0.0, 4 * macs);
}

double net_loss(hipStream_t st, const NetDev& N, int mt, const float* out, const float* tgt, float* gout, DBuf& scratch) {
    const int npix = N.npix();
    double* nd = (double*)scratch.ensure(sizeof(double) * 2 * mt);
    k_loss_cols<<<ceil_div(mt, 64), 64, 0, st>>>(npix, mt, out, tgt, nd, nd + mt);
    FH_LAUNCH_CHECK();
    k_loss_grad<<<ceil_div((size_t)npix * 2 * mt, 256), 256, 0, st>>>(npix, mt, out, tgt, nd + mt, gout);
    FH_LAUNCH_CHECK();
    std::vector<double> h(2 * mt);
    FH_HIP(hipMemcpyAsync(h.data(), nd, sizeof(double) * 2 * mt, hipMemcpyDeviceToHost, st));
    FH_HIP(hipStreamSynchronize(st));
    double l = 0.0;
    for (int c = 0; c < mt; ++c) l += h[c] / h[mt + c];
    return l / mt;
}

void net_adam(hipStream_t st, NetDev& N, const float* grad, float lr) {
    N.t += 1;
    k_adam<<<ceil_div(N.np, 256), 256, 0, st>>>(N.np, N.w, grad, N.mom, N.vel, N.wb, lr, 0.9f, 0.999f, 1e-8f, N.t);
    FH_LAUNCH_CHECK();
}

void net_sync_bf16(hipStream_t st, NetDev& N) {
    k_to_bf16<<<ceil_div(N.np, 256), 256, 0, st>>>(N.np, N.w, N.wb);
    FH_LAUNCH_CHECK();
}

void net_pack_diff(hipStream_t st, const NetDev& N, int m, int nsys, const float* o, const float* t, zd* D, zd* Tc) {
    const long tot = (long)N.npix() * m * nsys;
    k_net_pack_diff<<<ceil_div(tot, 256), 256, 0, st>>>(N.npix(), m, nsys, o, t, D, Tc);
    FH_LAUNCH_CHECK();
}

void net_grad_encode(hipStream_t st, const NetDev& N, int m, int nsys, const zd* G, const double* f, float* gout) {
    const long tot = (long)N.npix() * m * nsys;
    k_net_grad_encode<<<ceil_div(tot, 256), 256, 0, st>>>(N.npix(), m, nsys, G, f, gout);
    FH_LAUNCH_CHECK();
}

uint16_t host_f32_to_bf16(float f) { return f32_to_bf16(f); }

}  // namespace fh
