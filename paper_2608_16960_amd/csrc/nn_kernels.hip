// Companions of the projector on gfx950 (include/tspnn.h): total variation,
// Adam, and the layers of a small 3-D CNN on the spherical grid.
//
// 32 -> 32 convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16:
//   forward / input gradient: M = 16 voxels along azimuth, N = 16 output
//     channels, K = 32 input channels of one of the 27 taps; each lane loads
//     8 consecutive channels of one voxel (16 bytes, channels last);
//   weight gradient: M = 16 output channels, N = 16 input channels, K = 32
//     voxels of one azimuth row; rows of dz and the neighbour rows of x are
//     staged transposed in LDS so that each lane reads its 8 consecutive
//     voxels with one 16-byte LDS load (shifted by one azimuth: two 4-byte
//     neighbours and funnel shifts).
// MFMA lane layout used (16x16x32, wave64): lane l supplies A[l % 16][8 (l/16)
// .. +7] and B[8 (l/16) .. +7][l % 16] and receives D[4 (l/16) + i][l % 16],
// i = 0..3.
// All reductions (weight / bias gradients, TV value) write per-block partial
// sums and add them in a fixed order.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <string>

#include "tspnn.h"

namespace {

thread_local std::string g_err;

tspnn_status fail(tspnn_status s, const std::string &m) {
    g_err = m;
    return s;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int C = 32;  // channels of the hidden layers

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

struct Dims {
    int N, D0, D1, D2;
    __host__ __device__ __forceinline__ int64_t vox() const { return (int64_t)N * D0 * D1 * D2; }
};

// neighbour of voxel (n, i, j, k) at offset tap t; -1 when outside in r or e
__device__ __forceinline__ int64_t neighbour(const Dims &d, int n, int i, int j, int k, int t) {
    const int dr = t / 9 - 1, de = (t / 3) % 3 - 1, da = t % 3 - 1;
    const int ii = i + dr, jj = j + de;
    if (ii < 0 || ii >= d.D0 || jj < 0 || jj >= d.D1) return -1;
    int kk = k + da;
    kk = kk < 0 ? kk + d.D2 : (kk >= d.D2 ? kk - d.D2 : kk);
    return (((int64_t)n * d.D0 + ii) * d.D1 + jj) * d.D2 + kk;
}

__device__ __forceinline__ void unflatten(const Dims &d, int64_t p, int &n, int &i, int &j,
                                          int &k) {
    k = (int)(p % d.D2);
    int64_t q = p / d.D2;
    j = (int)(q % d.D1);
    q /= d.D1;
    i = (int)(q % d.D0);
    n = (int)(q / d.D0);
}

// ---------------------------------------------------------------- reductions

// out[j] = sum over b of part[b * stride + j] for j < count, b in increasing order
__global__ void k_reduce_parts(const float *part, int nb, int stride, int count, float *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    float s = 0.0f;
    for (int b = 0; b < nb; b++) s += part[(int64_t)b * stride + j];
    out[j] = s;
}

// out[g][j] = sum over b in [g * per, min(nb, (g + 1) * per)) of part[b * stride + j], in
// increasing b; the first stage of a two-stage fixed-order reduction.
__global__ void k_reduce_groups(const float *part, int nb, int stride, int count, int per,
                                float *out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (j >= count) return;
    const int b1 = min(nb, (g + 1) * per);
    float s = 0.0f;
    for (int b = g * per; b < b1; b++) s += part[(int64_t)b * stride + j];
    out[(int64_t)g * count + j] = s;
}

__device__ __forceinline__ float block_sum(float v, float *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) sh[w] = v;
    __syncthreads();
    float s = 0.0f;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += sh[i];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- TV

constexpr int kTvBlock = 256;

__device__ __forceinline__ float tv_term(float d, float eps) { return sqrtf(d * d + eps * eps); }

__global__ __launch_bounds__(kTvBlock) void k_tv(const float *rho, Dims d, float eps,
                                                 float *grad, float *part) {
    __shared__ float sh[4];
    const int64_t V = (int64_t)d.D0 * d.D1 * d.D2;
    const int b = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * kTvBlock + threadIdx.x;
    float val = 0.0f;
    if (p < V) {
        const float *r = rho + (int64_t)b * V;
        const int k = (int)(p % d.D2), j = (int)((p / d.D2) % d.D1), i = (int)(p / d.D2 / d.D1);
        const float c = r[p];
        const int64_t sr = (int64_t)d.D1 * d.D2, se = d.D2;
        float g = 0.0f;
        // own forward differences
        if (i + 1 < d.D0) {
            const float df = r[p + sr] - c, t = tv_term(df, eps);
            val += t;
            g -= df / t;
        }
        if (j + 1 < d.D1) {
            const float df = r[p + se] - c, t = tv_term(df, eps);
            val += t;
            g -= df / t;
        }
        {
            const int64_t q = (k + 1 < d.D2) ? p + 1 : p + 1 - d.D2;
            const float df = r[q] - c, t = tv_term(df, eps);
            val += t;
            g -= df / t;
        }
        // differences of the backward neighbours that involve this voxel
        if (i > 0) {
            const float df = c - r[p - sr];
            g += df / tv_term(df, eps);
        }
        if (j > 0) {
            const float df = c - r[p - se];
            g += df / tv_term(df, eps);
        }
        {
            const int64_t q = (k > 0) ? p - 1 : p - 1 + d.D2;
            const float df = c - r[q];
            g += df / tv_term(df, eps);
        }
        if (grad) grad[(int64_t)b * V + p] = g;
    }
    const float s = block_sum(val, sh);
    if (threadIdx.x == 0) part[(int64_t)b * gridDim.x + blockIdx.x] = s;
}

__global__ void k_tv_value(const float *part, int nblk, int B, float *value) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    float s = 0.0f;
    for (int i = 0; i < nblk; i++) s += part[(int64_t)b * nblk + i];
    value[b] = s;
}

// ---------------------------------------------------------------- Adam

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, float c1, float c2, uint16_t *pb) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i] + wd * p[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        p[i] = pi;
        if (pb) pb[i] = f2bf(pi);
    }
}

__global__ void k_to_bf16(const float *x, uint16_t *y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) y[i] = f2bf(x[i]);
}

__global__ void k_from_bf16(const uint16_t *x, float *y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) y[i] = bf2f(x[i]);
}

// ---------------------------------------------------------------- edge layers (VALU)

__global__ __launch_bounds__(256) void k_conv_in_fwd(const float *x, Dims d, const float *w,
                                                     const float *b, uint16_t *y) {
    __shared__ float ws[27 * C + C];
    for (int i = threadIdx.x; i < 27 * C; i += 256) ws[i] = w[i];
    if (threadIdx.x < C) ws[27 * C + threadIdx.x] = b[threadIdx.x];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= d.vox()) return;
    int n, i, j, k;
    unflatten(d, p, n, i, j, k);
    float xn[27];
#pragma unroll
    for (int t = 0; t < 27; t++) {
        const int64_t q = neighbour(d, n, i, j, k, t);
        xn[t] = q >= 0 ? x[q] : 0.0f;
    }
    u16x8 out[4];
#pragma unroll
    for (int o = 0; o < C; o++) {
        float a = ws[27 * C + o];
#pragma unroll
        for (int t = 0; t < 27; t++) a = fmaf(ws[t * C + o], xn[t], a);
        out[o >> 3][o & 7] = f2bf(fmaxf(a, 0.0f));
    }
    u16x8 *dst = (u16x8 *)(y + p * C);
#pragma unroll
    for (int q = 0; q < 4; q++) dst[q] = out[q];
}

__global__ __launch_bounds__(256) void k_conv_out_fwd(const uint16_t *x, Dims d, const float *w,
                                                      const float *b, const float *res,
                                                      float *out) {
    __shared__ float ws[27 * C];
    for (int i = threadIdx.x; i < 27 * C; i += 256) ws[i] = w[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= d.vox()) return;
    int n, i, j, k;
    unflatten(d, p, n, i, j, k);
    // eight partial sums (one per channel of a 16-byte group) keep the
    // multiply-adds independent; neighbours outside the grid read the voxel
    // itself and count zero
    float acc[8];
#pragma unroll
    for (int e = 0; e < 8; e++) acc[e] = 0.0f;
#pragma unroll 3
    for (int t = 0; t < 27; t++) {
        const int64_t q = neighbour(d, n, i, j, k, t);
        const float on = q >= 0 ? 1.0f : 0.0f;
        const u16x8 *src = (const u16x8 *)(x + (q >= 0 ? q : p) * C);
#pragma unroll
        for (int c8 = 0; c8 < 4; c8++) {
            const u16x8 v = src[c8];
#pragma unroll
            for (int e = 0; e < 8; e++)
                acc[e] = fmaf(ws[t * C + c8 * 8 + e] * on, bf2f(v[e]), acc[e]);
        }
    }
    float a = b[0] + (res ? res[p] : 0.0f);
#pragma unroll
    for (int e = 0; e < 8; e++) a += acc[e];
    out[p] = a;
}

// dz_in[q][i] = (sum_t w[t][i] dout[q - off(t)]) * (x[q][i] > 0)
__global__ __launch_bounds__(256) void k_conv_out_bwd_data(const uint16_t *x, const float *dout,
                                                           Dims d, const float *w,
                                                           uint16_t *dz) {
    __shared__ float ws[27 * C];
    for (int i = threadIdx.x; i < 27 * C; i += 256) ws[i] = w[i];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= d.vox()) return;
    int n, i, j, k;
    unflatten(d, p, n, i, j, k);
    float dn[27];
#pragma unroll
    for (int t = 0; t < 27; t++) {
        const int64_t q = neighbour(d, n, i, j, k, 26 - t);  // p - off(t) = p + off(26 - t)
        dn[t] = q >= 0 ? dout[q] : 0.0f;
    }
    const u16x8 *src = (const u16x8 *)(x + p * C);
    u16x8 *dst = (u16x8 *)(dz + p * C);
#pragma unroll
    for (int c8 = 0; c8 < 4; c8++) {
        const u16x8 xv = src[c8];
        u16x8 o;
#pragma unroll
        for (int e = 0; e < 8; e++) {
            float a = 0.0f;
#pragma unroll
            for (int t = 0; t < 27; t++) a = fmaf(ws[t * C + c8 * 8 + e], dn[t], a);
            o[e] = f2bf(bf2f(xv[e]) > 0.0f ? a : 0.0f);
        }
        dst[c8] = o;
    }
}

constexpr int kRowsPerBlk = 16;  // azimuth rows per block of the small weight gradients

// mode 0 (input layer):  part[blk][t*32+o] = sum_p dz[p][o] * xin[p + off(t)]
//                        part[blk][864+o]  = sum_p dz[p][o]
// mode 1 (output layer): part[blk][t*32+i] = sum_p dout[p] * x[p + off(t)][i]
//                        part[blk][864]    = sum_p dout[p]
// A block takes azimuth rows blk * kRowsPerBlk .. +kRowsPerBlk-1.  Thread
// (lr, dd, g) takes rows lr, lr + 7, ... of them, the neighbour row dd =
// (dr, de) of each and channels 8 g .. 8 g + 7: it walks the row's azimuths
// with the neighbour row's values at a - 1, a and a + 1 (circular) in
// registers, one new load per azimuth, and sums the three taps dd * 3 + da.
// The 7 row lanes are added in a fixed order through LDS.
constexpr int kRowLanes = 7;  // 7 x 36 threads

template <int MODE>
__global__ __launch_bounds__(256) void k_small_wgrad(const float *xin, const uint16_t *xb,
                                                     const uint16_t *dzb, const float *dout,
                                                     Dims d, float *part, int n_out) {
    __shared__ float sh[kRowLanes][28 * C];
    const int tid = threadIdx.x;
    const int lr = tid / 36, dd = (tid % 36) / 4, g = tid % 4;
    const int D2 = d.D2;
    float acc[3][8], bacc[8];
#pragma unroll
    for (int e = 0; e < 8; e++) {
        acc[0][e] = acc[1][e] = acc[2][e] = 0.0f;
        bacc[e] = 0.0f;
    }
    const int64_t rows = (int64_t)d.N * d.D0 * d.D1;
    const int64_t rend = min(rows, ((int64_t)blockIdx.x + 1) * kRowsPerBlk);
    for (int64_t row = (int64_t)blockIdx.x * kRowsPerBlk + lr; lr < kRowLanes && row < rend;
         row += kRowLanes) {
        const int i = (int)((row / d.D1) % d.D0), j = (int)(row % d.D1);
        const int n = (int)(row / d.D1 / d.D0);
        const int ii = i + dd / 3 - 1, jj = j + dd % 3 - 1;
        const bool ok = ii >= 0 && ii < d.D0 && jj >= 0 && jj < d.D1;
        const int64_t qb = ok ? (((int64_t)n * d.D0 + ii) * d.D1 + jj) * D2 : 0;
        const int64_t pb = row * D2;
        if (MODE == 1) {
            float xm[8], x0[8];
            const u16x8 vm = *reinterpret_cast<const u16x8 *>(xb + (qb + D2 - 1) * C + 8 * g);
            const u16x8 v0 = *reinterpret_cast<const u16x8 *>(xb + qb * C + 8 * g);
#pragma unroll
            for (int e = 0; e < 8; e++) {
                xm[e] = ok ? bf2f(vm[e]) : 0.0f;
                x0[e] = ok ? bf2f(v0[e]) : 0.0f;
            }
#pragma unroll 2
            for (int a = 0; a < D2; a++) {
                const int ap = a + 1 == D2 ? 0 : a + 1;
                const u16x8 vp = *reinterpret_cast<const u16x8 *>(xb + (qb + ap) * C + 8 * g);
                const float gs = dout[pb + a];
                bacc[0] += gs;
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const float xp = ok ? bf2f(vp[e]) : 0.0f;
                    acc[0][e] = fmaf(gs, xm[e], acc[0][e]);
                    acc[1][e] = fmaf(gs, x0[e], acc[1][e]);
                    acc[2][e] = fmaf(gs, xp, acc[2][e]);
                    xm[e] = x0[e];
                    x0[e] = xp;
                }
            }
        } else {
            float xm = ok ? xin[qb + D2 - 1] : 0.0f, x0 = ok ? xin[qb] : 0.0f;
#pragma unroll 2
            for (int a = 0; a < D2; a++) {
                const int ap = a + 1 == D2 ? 0 : a + 1;
                const float xp = ok ? xin[qb + ap] : 0.0f;
                const u16x8 gv = *reinterpret_cast<const u16x8 *>(dzb + (pb + a) * C + 8 * g);
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const float ge = bf2f(gv[e]);
                    bacc[e] += ge;
                    acc[0][e] = fmaf(ge, xm, acc[0][e]);
                    acc[1][e] = fmaf(ge, x0, acc[1][e]);
                    acc[2][e] = fmaf(ge, xp, acc[2][e]);
                }
                xm = x0;
                x0 = xp;
            }
        }
    }
    if (lr < kRowLanes) {
#pragma unroll
        for (int da = 0; da < 3; da++)
#pragma unroll
            for (int e = 0; e < 8; e++) sh[lr][(dd * 3 + da) * C + 8 * g + e] = acc[da][e];
        if (dd == 4) {  // the centre row carries the bias sums once
            if (MODE == 0) {
#pragma unroll
                for (int e = 0; e < 8; e++) sh[lr][27 * C + 8 * g + e] = bacc[e];
            } else if (g == 0) {
                sh[lr][27 * C] = bacc[0];
            }
        }
    }
    __syncthreads();
    for (int jo = tid; jo < n_out; jo += 256) {
        float v = 0.0f;
#pragma unroll
        for (int u = 0; u < kRowLanes; u++) v += sh[u][jo];
        part[(int64_t)blockIdx.x * n_out + jo] = v;
    }
}

// ---------------------------------------------------------------- 32 -> 32 on MFMA

// ring slot of r-row ii (ii >= -1)
__device__ __forceinline__ int ring_of(int ii) { return (ii + 3) % 3; }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
    return *reinterpret_cast<const bf16x8 *>(p);
}

// The same layer with its inputs staged in LDS.  A work item is a column of
// four e-rows (j0 .. j0 + 3) of one object and up to 64 azimuths a0 ..
// a0 + 63, walked along r over a chunk of `ilen` r-rows; wavefront w computes
// output row (i, j0 + w) at each step i.  The x rows a step reads are the
// 3 x 6 neighbour rows (r-rows i - 1 .. i + 1, e-rows j0 - 1 .. j0 + 4), each
// with one azimuth of circular halo on both sides (66 voxels of 64 bytes;
// rows outside the grid as zeros).  They sit in a ring of three r-slices of
// six rows in LDS (76 KB, two workgroups per CU), so a step brings in one new
// slice: the next step's slice is loaded into registers while this step's
// MFMAs run and stored after them.  An input row is fetched by 1.5 columns
// and (ilen + 2) / ilen steps, against 4 fetches with separately staged
// 2 x 2 tiles.  Per step a wavefront runs 27 taps of 8 MFMAs with no branch
// between them, the voxel fragments read from LDS and the weight fragments
// (which every workgroup shares, so they stay in cache) loaded, like the
// voxel fragments, one tap ahead.  Voxel q of a staged row keeps its four
// 16-byte channel groups c at position c ^ s(q), s(q) = ((q >> 1) ^ (q >> 3))
// & 3: 8 (16) consecutive voxels then cover all 32 (64) LDS banks, and a
// fragment's place is a per-lane offset plus a per-wavefront row base.
constexpr int kCols = 4;                       // e-rows per column
constexpr int kConvThreads = 64 * kCols;       // one wavefront per e-row
constexpr int kSliceRows = kCols + 2;          // x rows of one r-slice
constexpr int kStageVox = 66;                  // 64 azimuths + halo
constexpr int kConvItems = 512;                // work items a launch aims at (2 per CU)
// word 3 of a raw buffer resource: 32-bit data format, no swizzle
constexpr int kBufferDword3 = 0x00020000;

// place of channel group c of voxel q within a staged row (bf16 elements)
__device__ __forceinline__ int swz_off(int q, int c) {
    return (q * 4 + (c ^ (((q >> 1) ^ (q >> 3)) & 3))) * 8;
}

template <int EPI, int NT>
__device__ __forceinline__ void conv_walk(const uint16_t *__restrict__ x, const Dims &d,
                                          const uint16_t *__restrict__ w,
                                          const float *__restrict__ bias,
                                          const uint16_t *__restrict__ mask,
                                          uint16_t *__restrict__ y, uint16_t *xs, int n, int j0,
                                          int a0, int i0, int i1) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    constexpr int nq = NT * 16 + 2;  // staged voxels per row
    constexpr int kSlice = kSliceRows * nq * 4;  // 16-byte elements of one slice
    constexpr int KP = (kSlice + kConvThreads - 1) / kConvThreads;
    // Element e of the slice of r-row ii.  Every load of a slice is issued
    // before its first LDS store; an out-of-grid row loads element 0 (always
    // valid) and is zeroed at the store, so that no load sits behind a branch.
    auto load_el = [&](int ii, int u, u16x8 &v, bool &ok) {
        const int e = min(tid + u * kConvThreads, kSlice - 1);
        const int c = e & 3, q = (e >> 2) % nq, sl = (e >> 2) / nq;
        const int jj = j0 - 1 + sl;
        ok = ii >= 0 && ii < d.D0 && jj >= 0 && jj < d.D1;
        int a = a0 - 1 + q;
        a = a < 0 ? a + d.D2 : (a >= d.D2 ? a - d.D2 : a);
        const int64_t p = ok ? ((((int64_t)n * d.D0 + ii) * d.D1 + jj) * d.D2 + a) * C + 8 * c : 0;
        v = *reinterpret_cast<const u16x8 *>(x + p);
    };
    auto store_el = [&](int ii, int u, const u16x8 &v, bool ok) {
        const int e = tid + u * kConvThreads;
        const int c = e & 3, q = (e >> 2) % nq, sl = (e >> 2) / nq;
        const u16x8 z = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (e < kSlice)
            *reinterpret_cast<u16x8 *>(
                &xs[(ring_of(ii) * kSliceRows + sl) * kStageVox * C + swz_off(q, c)]) = ok ? v : z;
    };
    u16x8 pv[KP];
    bool pok[KP];
    // first step: slices i0 - 1 .. i0 + 1
    for (int s3 = 0; s3 < 3; s3++) {
#pragma unroll
        for (int u = 0; u < KP; u++) load_el(i0 - 1 + s3, u, pv[u], pok[u]);
#pragma unroll
        for (int u = 0; u < KP; u++) store_el(i0 - 1 + s3, u, pv[u], pok[u]);
    }
    const int j = j0 + wv;
    // weight fragments (output channels m and 16 + m) through a buffer
    // resource: one lane offset, the tap's offset in a scalar register
    const __amdgpu_buffer_rsrc_t wr =
        __builtin_amdgcn_make_buffer_rsrc((void *)w, (short)0, 27 * C * C * 2, kBufferDword3);
    const int wlo = (m * C + 8 * kq) * 2;  // bytes
    auto ldw = [&](int tap, int half) {
        return __builtin_bit_cast(
            bf16x8, __builtin_amdgcn_raw_buffer_load_b128(wr, wlo + half * 16 * C * 2,
                                                          tap * C * C * 2, 0));
    };
    // forward: this lane's eight biases (output channels 16 u + 4 kq .. + 3),
    // loaded once for the whole walk
    float bv[2][4];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
        for (int e = 0; e < 4; e++) bv[u][e] = EPI == 0 ? bias[16 * u + 4 * kq + e] : 0.0f;
    // input gradient: tap 0's weight fragments, the same at every step, held
    // for the walk (about 4% faster; the forward ran no faster with them)
    bf16x8 w00 = {}, w01 = {};
    if (EPI == 1) {
        w00 = ldw(0, 0);
        w01 = ldw(0, 1);
    }
    for (int i = i0; i < i1; i++) {
        if (i > i0) {
            __syncthreads();  // the previous step's reads are done
#pragma unroll
            for (int u = 0; u < KP; u++) store_el(i + 1, u, pv[u], pok[u]);
        }
        bf16x8 b0[2], b1[2];
        b0[0] = EPI == 1 ? w00 : ldw(0, 0);
        b1[0] = EPI == 1 ? w01 : ldw(0, 1);
        __syncthreads();
        if (i + 1 < i1) {  // slice i + 2, for the next step
#pragma unroll
            for (int u = 0; u < KP; u++) load_el(i + 2, u, pv[u], pok[u]);
        }
        if (j < d.D1) {  // uniform per wave
            const int64_t ob = (((int64_t)n * d.D0 + i) * d.D1 + j) * d.D2 + a0 + m;
            typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
            // input gradient: the ReLU mask of this step's outputs, loaded
            // before the taps so that it arrives while the MFMAs run
            u16x4 mkv[NT][2];
            if (EPI == 1) {
#pragma unroll
                for (int t = 0; t < NT; t++)
#pragma unroll
                    for (int u = 0; u < 2; u++)
                        mkv[t][u] = (a0 + 16 * t < d.D2)
                                        ? *reinterpret_cast<const u16x4 *>(
                                              mask + (ob + 16 * t) * C + 16 * u + 4 * kq)
                                        : u16x4{0, 0, 0, 0};
            }
            f32x4 acc[NT][2];
#pragma unroll
            for (int t = 0; t < NT; t++)
#pragma unroll
                for (int u = 0; u < 2; u++) acc[t][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            int slot[3];  // ring slots of r-rows i - 1, i, i + 1
#pragma unroll
            for (int dr = 0; dr < 3; dr++) slot[dr] = ring_of(i - 1 + dr);
            // voxel fragments of tap k (NT tiles of 16 azimuths)
            auto load_a = [&](int k, bf16x8 *av) {
                const int dr = k / 9, de = (k / 3) % 3, da = k % 3;  // offsets + 1
                const uint16_t *rp = xs + (slot[dr] * kSliceRows + wv + de) * kStageVox * C;
#pragma unroll
                for (int t = 0; t < NT; t++)
                    av[t] = *reinterpret_cast<const bf16x8 *>(rp + swz_off(16 * t + m + da, kq));
            };
            bf16x8 av[2][NT];
            load_a(0, av[0]);
            // both operands of the next tap are loaded while this tap's MFMAs run
#pragma unroll
            for (int tap = 0; tap < 27; tap++) {
                const int cur = tap & 1;
                if (tap + 1 < 27) {
                    b0[cur ^ 1] = ldw(tap + 1, 0);
                    b1[cur ^ 1] = ldw(tap + 1, 1);
                    load_a(tap + 1, av[cur ^ 1]);
                }
            // weights as the A operand and voxels as B: lane (m, kq) of tile
            // (t, u) holds output channels 16 u + 4 kq .. + 3 of voxel 16 t + m,
            // so its epilogue reads and writes 8 contiguous bytes
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    acc[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0[cur], av[cur][t], acc[t][0], 0, 0, 0);
                    acc[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b1[cur], av[cur][t], acc[t][1], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < NT; t++) {
                if (a0 + 16 * t >= d.D2) break;  // uniform
#pragma unroll
                for (int u = 0; u < 2; u++) {
                    const int o = 16 * u + 4 * kq;
                    const int64_t p = (ob + 16 * t) * C + o;
                    u16x4 out;
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        float v = acc[t][u][e];
                        if (EPI == 0) {
                            v = fmaxf(v + bv[u][e], 0.0f);
                        } else {
                            v = bf2f(mkv[t][u][e]) > 0.0f ? v : 0.0f;
                        }
                        out[e] = f2bf(v);
                    }
                    *reinterpret_cast<u16x4 *>(y + p) = out;
                }
            }
        }
    }
}

// Work items: (object, r-chunk, column of kCols e-rows, 64-azimuth chunk),
// the azimuth chunk fastest; one workgroup per item.
template <int EPI>
__global__ __launch_bounds__(kConvThreads, 2) void k_conv_lds(const uint16_t *__restrict__ x, Dims d,
                                                  int ilen, const uint16_t *__restrict__ w,
                                                  const float *__restrict__ bias,
                                                  const uint16_t *__restrict__ mask,
                                                  uint16_t *__restrict__ y) {
    __shared__ __attribute__((aligned(16))) uint16_t xs[3 * kSliceRows * kStageVox * C];
    const int nchunk = (d.D2 + 63) / 64, ncol = (d.D1 + kCols - 1) / kCols;
    const int nrch = (d.D0 + ilen - 1) / ilen;
    int64_t b = blockIdx.x;
    const int ac = (int)(b % nchunk);
    b /= nchunk;
    const int cj = (int)(b % ncol);
    b /= ncol;
    const int rc = (int)(b % nrch), n = (int)(b / nrch);
    const int a0 = ac * 64, j0 = cj * kCols, i0 = rc * ilen, i1 = min(d.D0, i0 + ilen);
    // D2 % 32 == 0: a last chunk of 32 azimuths runs as 64 (its halo and
    // upper half wrap around the row) and stores its lower half
    conv_walk<EPI, 4>(x, d, w, bias, mask, y, xs, n, j0, a0, i0, i1);
}

constexpr int kMaxD2 = 128;  // widest azimuth row of the MFMA layers

// Weight gradient of a 32 -> 32 layer.  A work item is a column of two
// e-rows (j0, j0 + 1) of one object, walked along r over a chunk of
// `ilen` r-rows; a workgroup takes items blockIdx.x, + gridDim.x, ...  The
// x rows an output row meets are the 3 x 4 neighbour rows (r-rows i - 1 ..
// i + 1, e-rows j0 - 1 .. j0 + 2); they sit in a ring of three r-slices of
// four e-rows in LDS, so a step along r brings in one new slice (4 rows) and
// the two dz rows; the first step of an item stages three slices.  The next
// step's slice and dz rows are loaded into registers while this step's
// products run, and stored to LDS after them.  Rows are staged transposed
// to [channel][azimuth] (rows outside the grid as zeros).  A staged x row
// keeps azimuth a at position a + 8, with a - 1 of a = 0 at 7 and a + 1 of
// a = D2 - 1 at D2 + 8, so that the operand of shift 0 is one aligned
// 16-byte read and those of shifts -1 and +1 follow from it and two 4-byte
// neighbours by funnel shifts.  Staging stores pack two azimuths of one
// channel into 4 bytes; channel rows have an odd number of 16-byte units,
// so the 16 rows an MFMA reads fall in different banks.  Wavefront w owns
// output channels 16 (w >> 1) .. +15 and input channels 16 (w & 1) .. +15 of
// all 27 taps; its sums stay in registers until the workgroup's last item,
// then go out as its partial sums.
constexpr int kWRows = 2;                  // e-rows per column
constexpr int kWStage = 3 * (kWRows + 2);  // x rows in the ring: 3 slices of 4
constexpr int kWPart = 27 * C * C + C;     // a workgroup's partial sums: weights, then bias
constexpr int kWGroups = 32;               // first-stage groups of their reduction

__device__ __forceinline__ uint32_t pack_bf16x2(uint16_t lo, uint16_t hi) {
    return (uint32_t)lo | ((uint32_t)hi << 16);
}

template <int D2>
__global__ __launch_bounds__(256, D2 <= 64 ? 2 : 1) void k_conv_wgrad_tiled(const uint16_t *__restrict__ x,
                                                          const uint16_t *__restrict__ dz, Dims d,
                                                          int ilen, float *__restrict__ part) {
    extern __shared__ __attribute__((aligned(16))) uint16_t lds[];
    constexpr int sx = D2 + 24, sz = D2 + 8;  // channel-row strides (bf16 elements)
    // staging elements: an x element is two azimuths (2 pi - 2, 2 pi - 1 mod D2,
    // at positions 6 + 2 pi) of 8 channels of one row; a dz element two
    // azimuths (2 pi, 2 pi + 1) of 8 channels
    constexpr int npx = D2 / 2 + 2, npz = D2 / 2;
    constexpr int kSlice = (kWRows + 2) * 4 * npx, kZ = kWRows * 4 * npz;
    constexpr int KX = (kSlice + 255) / 256, KZ = (kZ + 255) / 256;
    constexpr int nkb = D2 / 32;
    uint16_t *xT = lds;                     // [kWStage][C][sx]: row 4 ring_of(ii) + (jj - j0 + 1)
    uint16_t *zT = lds + kWStage * C * sx;  // [kWRows][C][sz]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int ot = wv >> 1, ct = wv & 1;  // output / input channel tiles
    const int njb = (d.D1 + kWRows - 1) / kWRows;
    const int nch = (d.D0 + ilen - 1) / ilen;
    const int64_t nitems = (int64_t)d.N * njb * nch;
    f32x4 acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;  // bias gradient: wavefronts of input tile 0 add up their dz operands
    const u16x8 zero8 = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int ch = (int)(item % nch);
        const int64_t col = item / nch;
        const int j0 = (int)(col % njb) * kWRows, n = (int)(col / njb);
        const int i0 = ch * ilen, i1 = min(d.D0, i0 + ilen);
        // element e of the x slice of r-row ii, and its LDS place
        auto load_x = [&](int ii, int e, u16x8 &v0, u16x8 &v1) {
            const int pi = e % npx, c8 = ((e / npx) & 3) * 8, sl = e / npx / 4;
            const int jj = j0 - 1 + sl;
            v0 = zero8;
            v1 = zero8;
            if (ii >= 0 && ii < d.D0 && jj >= 0 && jj < d.D1) {
                int a = 2 * pi - 2;
                a = a < 0 ? a + D2 : (a >= D2 ? a - D2 : a);
                const int a1 = a + 1 == D2 ? 0 : a + 1;
                const int64_t rb = (((int64_t)n * d.D0 + ii) * d.D1 + jj) * D2;
                v0 = *reinterpret_cast<const u16x8 *>(x + (rb + a) * C + c8);
                v1 = *reinterpret_cast<const u16x8 *>(x + (rb + a1) * C + c8);
            }
        };
        auto store_x = [&](int ii, int e, const u16x8 &v0, const u16x8 &v1) {
            const int pi = e % npx, c8 = ((e / npx) & 3) * 8, sl = e / npx / 4;
            const int row = ring_of(ii) * (kWRows + 2) + sl;
            uint32_t *dst = reinterpret_cast<uint32_t *>(xT + (row * C + c8) * sx + 6 + 2 * pi);
#pragma unroll
            for (int q = 0; q < 8; q++) dst[q * (sx / 2)] = pack_bf16x2(v0[q], v1[q]);
        };
        // element e of the dz rows (ii, j0), (ii, j0 + 1)
        auto load_z = [&](int ii, int e, u16x8 &v0, u16x8 &v1) {
            const int pi = e % npz, c8 = ((e / npz) & 3) * 8, r = e / npz / 4;
            v0 = zero8;
            v1 = zero8;
            if (j0 + r < d.D1) {
                const int64_t rb = (((int64_t)n * d.D0 + ii) * d.D1 + j0 + r) * D2;
                v0 = *reinterpret_cast<const u16x8 *>(dz + (rb + 2 * pi) * C + c8);
                v1 = *reinterpret_cast<const u16x8 *>(dz + (rb + 2 * pi + 1) * C + c8);
            }
        };
        auto store_z = [&](int e, const u16x8 &v0, const u16x8 &v1) {
            const int pi = e % npz, c8 = ((e / npz) & 3) * 8, r = e / npz / 4;
            uint32_t *dst = reinterpret_cast<uint32_t *>(zT + (r * C + c8) * sz + 2 * pi);
#pragma unroll
            for (int q = 0; q < 8; q++) dst[q * (sz / 2)] = pack_bf16x2(v0[q], v1[q]);
        };
        __syncthreads();  // the previous item's reads are done
        // first step: slices i0 - 1 .. i0 + 1 and dz of r-row i0
        for (int e = tid; e < 3 * kSlice; e += 256) {
            u16x8 v0, v1;
            load_x(i0 - 1 + e / kSlice, e % kSlice, v0, v1);
            store_x(i0 - 1 + e / kSlice, e % kSlice, v0, v1);
        }
        for (int e = tid; e < kZ; e += 256) {
            u16x8 v0, v1;
            load_z(i0, e, v0, v1);
            store_z(e, v0, v1);
        }
        u16x8 px0[KX], px1[KX], pz0[KZ], pz1[KZ];  // the next step's rows in flight
        for (int i = i0; i < i1; i++) {
            if (i > i0) {
                __syncthreads();  // the previous step's reads are done
#pragma unroll
                for (int k = 0; k < KX; k++)
                    if (tid + 256 * k < kSlice) store_x(i + 1, tid + 256 * k, px0[k], px1[k]);
#pragma unroll
                for (int k = 0; k < KZ; k++)
                    if (tid + 256 * k < kZ) store_z(tid + 256 * k, pz0[k], pz1[k]);
            }
            __syncthreads();
            if (i + 1 < i1) {  // slice i + 2 and dz of r-row i + 1, for the next step
#pragma unroll
                for (int k = 0; k < KX; k++)
                    if (tid + 256 * k < kSlice) load_x(i + 2, tid + 256 * k, px0[k], px1[k]);
#pragma unroll
                for (int k = 0; k < KZ; k++)
                    if (tid + 256 * k < kZ) load_z(i + 1, tid + 256 * k, pz0[k], pz1[k]);
            }
            int slot[3];  // ring slots of r-rows i - 1, i, i + 1
#pragma unroll
            for (int dr = 0; dr < 3; dr++) slot[dr] = ring_of(i - 1 + dr);
#pragma unroll
            for (int kb = 0; kb < nkb; kb++) {
                const int a = 32 * kb + 8 * kq;
                // dz operands of both e-rows (a row beyond the grid was staged
                // as zeros and adds nothing)
                const u16x8 A0u = *reinterpret_cast<const u16x8 *>(zT + (16 * ot + m) * sz + a);
                const u16x8 A1u = *reinterpret_cast<const u16x8 *>(zT + (C + 16 * ot + m) * sz + a);
                const bf16x8 A0 = __builtin_bit_cast(bf16x8, A0u);
                const bf16x8 A1 = __builtin_bit_cast(bf16x8, A1u);
                if (ct == 0) {  // uniform per wavefront
#pragma unroll
                    for (int e = 0; e < 8; e++) bsum += bf2f(A0u[e]) + bf2f(A1u[e]);
                }
                // the 12 staged x rows (3 r-slices x 4 e-rows); x row sl of a
                // slice meets dz row 0 at e-offset sl and dz row 1 at sl - 1,
                // so each row is read once for both.  The next row's reads are
                // issued before this row's products.
                typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
                const uint16_t *xb = xT + (16 * ct + m) * sx + a + 8;
                auto load_row = [&](int q, u32x4 &c, uint32_t &lo, uint32_t &hi) {
                    const uint16_t *bp = xb + (slot[q >> 2] * (kWRows + 2) + (q & 3)) * C * sx;
                    c = *reinterpret_cast<const u32x4 *>(bp);
                    lo = *reinterpret_cast<const uint32_t *>(bp - 2);
                    hi = *reinterpret_cast<const uint32_t *>(bp + 8);
                };
                u32x4 c;
                uint32_t lo, hi;
                load_row(0, c, lo, hi);
#pragma unroll
                for (int q = 0; q < 3 * (kWRows + 2); q++) {
                    u32x4 cn = c;
                    uint32_t lon = lo, hin = hi;
                    if (q + 1 < 3 * (kWRows + 2)) load_row(q + 1, cn, lon, hin);
                    const uint32_t f0 = __builtin_amdgcn_alignbit(c[0], lo, 16);
                    const uint32_t f1 = __builtin_amdgcn_alignbit(c[1], c[0], 16);
                    const uint32_t f2 = __builtin_amdgcn_alignbit(c[2], c[1], 16);
                    const uint32_t f3 = __builtin_amdgcn_alignbit(c[3], c[2], 16);
                    const uint32_t f4 = __builtin_amdgcn_alignbit(hi, c[3], 16);
                    const bf16x8 bm = __builtin_bit_cast(bf16x8, u32x4{f0, f1, f2, f3});
                    const bf16x8 b0 = __builtin_bit_cast(bf16x8, c);
                    const bf16x8 bpl = __builtin_bit_cast(bf16x8, u32x4{f1, f2, f3, f4});
                    const int dr = q / (kWRows + 2), sl = q % (kWRows + 2);
                    if (sl <= 2) {  // dz row 0, e-offset sl - 1
                        const int t0 = (dr * 3 + sl) * 3;
                        acc[t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, bm, acc[t0], 0, 0, 0);
                        acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, b0, acc[t0 + 1], 0, 0, 0);
                        acc[t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, bpl, acc[t0 + 2], 0, 0, 0);
                    }
                    if (sl >= 1) {  // dz row 1, e-offset sl - 2
                        const int t0 = (dr * 3 + sl - 1) * 3;
                        acc[t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, bm, acc[t0], 0, 0, 0);
                        acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, b0, acc[t0 + 1], 0, 0, 0);
                        acc[t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, bpl, acc[t0 + 2], 0, 0, 0);
                    }
                    c = cn;
                    lo = lon;
                    hi = hin;
                }
            }
        }
    }
    // partial sums: row blk of part holds [tap][o][i], then the bias [o]
    float *pb = part + (int64_t)blockIdx.x * kWPart;
#pragma unroll
    for (int t = 0; t < 27; t++)
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int o = 16 * ot + 4 * kq + e, ci = 16 * ct + m;
            pb[((int64_t)t * C + o) * C + ci] = acc[t][e];
        }
    if (ct == 0) {  // lanes m, m + 16, m + 32, m + 48 hold channel 16 ot + m
        bsum += __shfl_xor(bsum, 16, 64);
        bsum += __shfl_xor(bsum, 32, 64);
        if (kq == 0) pb[27 * C * C + 16 * ot + m] = bsum;
    }
}

// The weight-gradient partial rows summed in a fixed order, in two stages.
// Stage 1: tmp[g] = the sum of rows g * per .. min(nb, (g + 1) * per) - 1, in
// increasing order, per 16-byte column.
__global__ __launch_bounds__(256) void k_wgrad_groups(const f32x4 *__restrict__ part, int nb,
                                                      int per, f32x4 *__restrict__ tmp) {
    constexpr int n4 = kWPart / 4;
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n4) return;
    const int b1 = min(nb, (int)(blockIdx.y + 1) * per);
    int b = blockIdx.y * per;
    f32x4 s = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (; b + 8 <= b1; b += 8) {  // eight loads in flight, added in order
        f32x4 v[8];
#pragma unroll
        for (int k = 0; k < 8; k++) v[k] = part[(int64_t)(b + k) * n4 + j];
#pragma unroll
        for (int k = 0; k < 8; k++) s += v[k];
    }
    for (; b < b1; b++) s += part[(int64_t)b * n4 + j];
    tmp[(int64_t)blockIdx.y * n4 + j] = s;
}

// Stage 2: the kWGroups group sums of a column, in order: four threads take
// eight groups each, then thread 0 of the four adds their sums in order.
// Columns below 27 C C go to dw, the rest to db (skipped when db is null).
__global__ __launch_bounds__(256) void k_wgrad_final(const f32x4 *__restrict__ tmp,
                                                     float *__restrict__ dw,
                                                     float *__restrict__ db) {
    constexpr int n4 = kWPart / 4, per = kWGroups / 4;
    const int j = blockIdx.x * 64 + (threadIdx.x >> 2), q = threadIdx.x & 3;
    f32x4 s = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    if (j < n4) {
        f32x4 v[per];
#pragma unroll
        for (int k = 0; k < per; k++) v[k] = tmp[(int64_t)(q * per + k) * n4 + j];
#pragma unroll
        for (int k = 0; k < per; k++) s += v[k];
    }
    f32x4 t[4];
#pragma unroll
    for (int k = 0; k < 4; k++)
#pragma unroll
        for (int e = 0; e < 4; e++) t[k][e] = __shfl(s[e], (threadIdx.x & ~3) + k, 64);
    if (j >= n4 || q != 0) return;
    const f32x4 r = ((t[0] + t[1]) + t[2]) + t[3];
    const int e0 = 4 * j;  // dw and db need only 4-byte alignment
    if (e0 < 27 * C * C) {
#pragma unroll
        for (int e = 0; e < 4; e++) dw[e0 + e] = r[e];
    } else if (db) {
#pragma unroll
        for (int e = 0; e < 4; e++) db[e0 - 27 * C * C + e] = r[e];
    }
}

size_t wgrad_lds_bytes(int D2) {
    return sizeof(uint16_t) * ((size_t)kWStage * C * (D2 + 24) + (size_t)kWRows * C * (D2 + 8));
}

__global__ void k_flip(const uint16_t *w, uint16_t *wt) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 27 * C * C) return;
    const int t = e / (C * C), i = (e / C) % C, o = e % C;
    wt[e] = w[((26 - t) * C + o) * C + i];  // wt[t][i][o]
}

inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }
// Elementwise kernels over caller-sized arrays stride over their items and
// take at most 2^23 workgroups of 256 (one dispatch holds fewer than 2^32
// work-items), or fewer from the environment variable TSP_MAX_BLOCKS (read
// once per process), so that tests can make the striding run at small sizes.
inline unsigned nblk_strided(int64_t n) {
    static const int64_t cap = [] {
        const char *s = std::getenv("TSP_MAX_BLOCKS");
        const long long v = s ? std::atoll(s) : 0;
        return (v > 0 && v < ((int64_t)1 << 23)) ? (int64_t)v : ((int64_t)1 << 23);
    }();
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

// ------------------------------------------------ per-object vector kernels
//
// Objects are rows of n floats.  A reduction over a row runs in two fixed
// stages: blocks of kVecChunk consecutive elements (a fixed-order block sum),
// then the chunks of each row in increasing order (reduce_parts), so results
// do not depend on timing.
constexpr int kVecChunk = 8192;

// OP 0: diff = f - y (when diff is not null), part = sum of diff^2;
// OP 1: part = sum of a * b.  part[chunk][object].
template <int OP>
__global__ __launch_bounds__(256) void k_vec_part(const float *__restrict__ a,
                                                  const float *__restrict__ b, int64_t n,
                                                  float *__restrict__ diff,
                                                  float *__restrict__ part) {
    __shared__ float sh[4];
    const int k = blockIdx.x, o = blockIdx.y;
    const int64_t lo = (int64_t)k * kVecChunk;
    const int64_t hi = min(lo + (int64_t)kVecChunk, n);
    const int64_t off = (int64_t)o * n;
    float acc = 0.0f;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
        if (OP == 0) {
            const float d = b[off + i] - a[off + i];
            if (diff) diff[off + i] = d;
            acc = fmaf(d, d, acc);
        } else {
            acc = fmaf(a[off + i], b[off + i], acc);
        }
    }
    const float t = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)k * gridDim.y + o] = t;
}

// out[o] = sums[o] where active[o] (every o when active is null)
__global__ void k_store_masked(const float *sums, const int32_t *active, int B, float *out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o < B && (!active || active[o])) out[o] = sums[o];
}

// x[o][i] += alpha * a[o][i] for active o
__global__ void k_axpy(float *x, const float *a, float alpha, int64_t n, int64_t total,
                       const int32_t *active) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        if (!active || active[i / n]) x[i] = fmaf(alpha, a[i], x[i]);
}

__global__ void k_scale(const float *src, float alpha, int64_t n, float *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) dst[i] = alpha * src[i];
}



// Workgroups of the weight gradient: two per CU (one wavefront per SIMD left
// the LDS transposes and barriers of each row unhidden: 0.67 ms at batch 8 of
// 64x32x64 against 0.46 ms with 512); more only add partial sums to reduce.
int wgrad_blocks(int64_t rows) { return (int)(rows < 512 ? rows : 512); }

constexpr int kRedGroups = 16;  // first-stage groups of the partial reductions

// out[j] = sum over the nb partial rows part[b * stride + j], j < count, in a
// fixed order: kRedGroups groups of consecutive rows summed in parallel into
// tmp [kRedGroups][count], then the group sums.
void reduce_parts(const float *part, int nb, int stride, int count, float *out, float *tmp,
                  hipStream_t st) {
    if (nb <= 2 * kRedGroups) {
        hipLaunchKernelGGL(k_reduce_parts, dim3(nblk(count, 256)), dim3(256), 0, st, part, nb,
                           stride, count, out);
        return;
    }
    const int per = (nb + kRedGroups - 1) / kRedGroups;
    hipLaunchKernelGGL(k_reduce_groups, dim3(nblk(count, 256), kRedGroups), dim3(256), 0, st, part,
                       nb, stride, count, per, tmp);
    hipLaunchKernelGGL(k_reduce_parts, dim3(nblk(count, 256)), dim3(256), 0, st, tmp, kRedGroups,
                       count, count, out);
}

bool aligned16(const void *p) { return (uintptr_t)p % 16 == 0; }

bool dims_ok(int N, int D0, int D1, int D2) { return N > 0 && D0 > 0 && D1 > 0 && D2 > 0; }

tspnn_status hipret(hipError_t e, const char *what) {
    if (e != hipSuccess) return fail(TSPNN_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return TSPNN_OK;
}

// work items of k_conv_lds: columns (object, e-row block, azimuth chunk) cut
// along r into chunks of ilen r-rows, so that there are about kConvItems
struct ConvPlan {
    int ilen;
    unsigned items;
};
ConvPlan conv_plan(const Dims &d) {
    const int64_t cols = (int64_t)d.N * ((d.D1 + kCols - 1) / kCols) * ((d.D2 + 63) / 64);
    const int64_t nrch =
        std::max<int64_t>(1, std::min<int64_t>(d.D0, (kConvItems + cols - 1) / cols));
    const int ilen = (int)((d.D0 + nrch - 1) / nrch);
    return {ilen, (unsigned)(cols * ((d.D0 + ilen - 1) / ilen))};
}

tspnn_status mfma_dims(int N, int D0, int D1, int D2) {
    if (!dims_ok(N, D0, D1, D2)) return fail(TSPNN_E_INVALID, "dimensions must be positive");
    if (D2 % 32 != 0 || D2 > kMaxD2)
        return fail(TSPNN_E_UNSUPPORTED, "MFMA layers need D2 % 32 == 0 and D2 <= 128");
    return TSPNN_OK;
}

// Streaming copy and read of 16-byte elements with non-temporal loads and
// stores: a measurement of the HBM rate a plain stream reaches on this
// device, for the roofline of the projector kernels.  Each thread keeps
// kStreamUnroll independent 16-byte loads in flight per iteration of a
// grid-stride loop over the whole array.
constexpr int kStreamUnroll = 4;

__global__ __launch_bounds__(256) void k_stream_copy(const f32x4 *__restrict__ src,
                                                      f32x4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + (kStreamUnroll - 1) * stride < n; i += kStreamUnroll * stride) {
        f32x4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; u++) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kStreamUnroll; u++) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// partial[block] = sum of the elements the block read (keeps the loads live)
__global__ __launch_bounds__(256) void k_stream_read(const f32x4 *__restrict__ src, int64_t n,
                                                      float *__restrict__ partial) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    for (; i + (kStreamUnroll - 1) * stride < n; i += kStreamUnroll * stride) {
        f32x4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; u++) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < kStreamUnroll; u++) acc += v[u];
    }
    for (; i < n; i += stride) acc += __builtin_nontemporal_load(src + i);
    float t = acc[0] + acc[1] + acc[2] + acc[3];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    __shared__ float ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

}  // namespace

extern "C" {

const char *tspnn_last_error(void) { return g_err.c_str(); }

size_t tspnn_tv_workspace(int32_t B, int64_t V) {
    return sizeof(float) * (size_t)B * (size_t)((V + kTvBlock - 1) / kTvBlock) + 64;
}

tspnn_status tspnn_tv(const float *rho, int32_t B, int32_t D0, int32_t D1, int32_t D2, float eps,
                      float *value, float *grad, void *work, void *stream) {
    g_err.clear();
    if (!rho || !value || !work || B < 1 || !dims_ok(1, D0, D1, D2))
        return fail(TSPNN_E_INVALID, "tspnn_tv: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    const int64_t V = (int64_t)D0 * D1 * D2;
    const unsigned nb = nblk(V, kTvBlock);
    Dims d{1, D0, D1, D2};
    hipLaunchKernelGGL(k_tv, dim3(nb, B), dim3(kTvBlock), 0, st, rho, d, eps, grad, (float *)work);
    hipLaunchKernelGGL(k_tv_value, dim3(nblk(B, 64)), dim3(64), 0, st, (const float *)work, (int)nb,
                       B, value);
    return hipret(hipGetLastError(), "tspnn_tv");
}

tspnn_status tspnn_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                        float beta1, float beta2, float eps, float weight_decay, int32_t step,
                        uint16_t *p_bf16, void *stream) {
    g_err.clear();
    if (!p || !g || !m || !v || n < 0 || step < 1)
        return fail(TSPNN_E_INVALID, "tspnn_adam: bad arguments");
    if (n == 0) return TSPNN_OK;
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk_strided(n)), dim3(256), 0, (hipStream_t)stream, p, g, m,
                       v, n, lr, beta1, beta2, eps, weight_decay, c1, c2, p_bf16);
    return hipret(hipGetLastError(), "tspnn_adam");
}

tspnn_status tspnn_to_bf16(const float *x, uint16_t *y, int64_t n, void *stream) {
    g_err.clear();
    if (!x || !y || n < 0) return fail(TSPNN_E_INVALID, "tspnn_to_bf16: bad arguments");
    if (n == 0) return TSPNN_OK;
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk_strided(n)), dim3(256), 0, (hipStream_t)stream, x, y,
                       n);
    return hipret(hipGetLastError(), "tspnn_to_bf16");
}

tspnn_status tspnn_from_bf16(const uint16_t *x, float *y, int64_t n, void *stream) {
    g_err.clear();
    if (!x || !y || n < 0) return fail(TSPNN_E_INVALID, "tspnn_from_bf16: bad arguments");
    if (n == 0) return TSPNN_OK;
    hipLaunchKernelGGL(k_from_bf16, dim3(nblk_strided(n)), dim3(256), 0, (hipStream_t)stream, x, y,
                       n);
    return hipret(hipGetLastError(), "tspnn_from_bf16");
}

size_t tspnn_conv_workspace(int32_t N, int32_t D0, int32_t D1, int32_t D2) {
    const int64_t rows = (int64_t)N * D0 * D1;
    const int64_t wb = wgrad_blocks(rows);
    // 32 -> 32 layers: partial rows (weights and bias) and their group sums;
    // edge layers: partials and group sums
    const size_t a = sizeof(float) * (size_t)(wb + kWGroups) * kWPart;
    const int64_t rblk = (rows + kRowsPerBlk - 1) / kRowsPerBlk;
    const size_t b = sizeof(float) * ((size_t)rblk + kRedGroups) * (27 * C + C);
    return (a > b ? a : b) + 256;
}

tspnn_status tspnn_conv_in_fwd(const float *x, int32_t N, int32_t D0, int32_t D1, int32_t D2,
                               const float *w, const float *b, uint16_t *y, void *stream) {
    g_err.clear();
    if (!x || !w || !b || !y || !dims_ok(N, D0, D1, D2))
        return fail(TSPNN_E_INVALID, "tspnn_conv_in_fwd: bad arguments");
    Dims d{N, D0, D1, D2};
    hipLaunchKernelGGL(k_conv_in_fwd, dim3(nblk(d.vox(), 256)), dim3(256), 0, (hipStream_t)stream,
                       x, d, w, b, y);
    return hipret(hipGetLastError(), "tspnn_conv_in_fwd");
}

tspnn_status tspnn_conv_fwd(const uint16_t *x, int32_t N, int32_t D0, int32_t D1, int32_t D2,
                            const uint16_t *w, const float *b, uint16_t *y, void *stream) {
    g_err.clear();
    if (!x || !w || !b || !y) return fail(TSPNN_E_INVALID, "tspnn_conv_fwd: NULL argument");
    if (!aligned16(x) || !aligned16(w) || !aligned16(y))
        return fail(TSPNN_E_INVALID, "tspnn_conv_fwd: bfloat16 arrays must be 16-byte aligned");
    tspnn_status s = mfma_dims(N, D0, D1, D2);
    if (s != TSPNN_OK) return s;
    Dims d{N, D0, D1, D2};
    const ConvPlan pl = conv_plan(d);
    hipLaunchKernelGGL(k_conv_lds<0>, dim3(pl.items), dim3(kConvThreads), 0, (hipStream_t)stream,
                       x, d, pl.ilen, w, b, (const uint16_t *)nullptr, y);
    return hipret(hipGetLastError(), "tspnn_conv_fwd");
}

tspnn_status tspnn_conv_bwd_data(const uint16_t *dz_out, int32_t N, int32_t D0, int32_t D1,
                                 int32_t D2, const uint16_t *w, const uint16_t *act_in,
                                 uint16_t *dz_in, void *stream) {
    g_err.clear();
    if (!dz_out || !w || !act_in || !dz_in)
        return fail(TSPNN_E_INVALID, "tspnn_conv_bwd_data: NULL argument");
    if (!aligned16(dz_out) || !aligned16(w) || !aligned16(act_in) || !aligned16(dz_in))
        return fail(TSPNN_E_INVALID,
                    "tspnn_conv_bwd_data: bfloat16 arrays must be 16-byte aligned");
    tspnn_status s = mfma_dims(N, D0, D1, D2);
    if (s != TSPNN_OK) return s;
    Dims d{N, D0, D1, D2};
    const ConvPlan pl = conv_plan(d);
    hipLaunchKernelGGL(k_conv_lds<1>, dim3(pl.items), dim3(kConvThreads), 0, (hipStream_t)stream,
                       dz_out, d, pl.ilen, w, (const float *)nullptr, act_in, dz_in);
    return hipret(hipGetLastError(), "tspnn_conv_bwd_data");
}

tspnn_status tspnn_conv_bwd_weight(const uint16_t *x, const uint16_t *dz, int32_t N, int32_t D0,
                                   int32_t D1, int32_t D2, float *dw, float *db, void *work,
                                   void *stream) {
    g_err.clear();
    if (!x || !dz || !dw || !work) return fail(TSPNN_E_INVALID, "tspnn_conv_bwd_weight: NULL");
    if (!aligned16(work) || !aligned16(x) || !aligned16(dz))
        return fail(TSPNN_E_INVALID,
                    "tspnn_conv_bwd_weight: x, dz and work must be 16-byte aligned");
    tspnn_status s = mfma_dims(N, D0, D1, D2);
    if (s != TSPNN_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    Dims d{N, D0, D1, D2};
    // columns of two e-rows, cut along r into chunks so that there are about
    // 512 work items; never more workgroups than the workspace holds partial
    // sums for (wgrad_blocks of the row count)
    const int64_t cols = (int64_t)N * ((D1 + kWRows - 1) / kWRows);
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(D0, (512 + cols - 1) / cols));
    const int ilen = (int)((D0 + nch - 1) / nch);
    const int64_t items = cols * ((D0 + ilen - 1) / ilen);
    const int nb = wgrad_blocks(items);
    float *part = (float *)work;
    const size_t lds = wgrad_lds_bytes(D2);
    using wgrad_fn = void (*)(const uint16_t *, const uint16_t *, Dims, int, float *);
    const wgrad_fn fns[4] = {k_conv_wgrad_tiled<32>, k_conv_wgrad_tiled<64>,
                             k_conv_wgrad_tiled<96>, k_conv_wgrad_tiled<128>};
    // dynamic LDS above the default needs opting in, once per device
    static bool lds_enabled[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hipret(e, "tspnn_conv_bwd_weight");
    if (dev < 0 || dev >= 64 || !lds_enabled[dev]) {
        for (int k = 0; k < 4; k++) {
            e = hipFuncSetAttribute((const void *)fns[k],
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)wgrad_lds_bytes(32 * (k + 1)));
            if (e != hipSuccess) return hipret(e, "tspnn_conv_bwd_weight (LDS size)");
        }
        if (dev >= 0 && dev < 64) lds_enabled[dev] = true;
    }
    // workspace: nb partial rows, then kWGroups group sums (tspnn_conv_workspace
    // sizes it)
    hipLaunchKernelGGL(fns[D2 / 32 - 1], dim3(nb), dim3(256), lds, st, x, dz, d, ilen, part);
    float *tmp = part + (int64_t)nb * kWPart;
    const int per = (nb + kWGroups - 1) / kWGroups;
    hipLaunchKernelGGL(k_wgrad_groups, dim3(nblk(kWPart / 4, 256), kWGroups), dim3(256), 0, st,
                       (const f32x4 *)part, nb, per, (f32x4 *)tmp);
    hipLaunchKernelGGL(k_wgrad_final, dim3(nblk(kWPart / 4, 64)), dim3(256), 0, st,
                       (const f32x4 *)tmp, dw, db);
    return hipret(hipGetLastError(), "tspnn_conv_bwd_weight");
}

tspnn_status tspnn_conv_in_bwd_weight(const float *x, const uint16_t *dz, int32_t N, int32_t D0,
                                      int32_t D1, int32_t D2, float *dw, float *db, void *work,
                                      void *stream) {
    g_err.clear();
    if (!x || !dz || !dw || !db || !work || !dims_ok(N, D0, D1, D2))
        return fail(TSPNN_E_INVALID, "tspnn_conv_in_bwd_weight: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    Dims d{N, D0, D1, D2};
    const int nc = (int)(((int64_t)N * D0 * D1 + kRowsPerBlk - 1) / kRowsPerBlk);
    const int n_out = 27 * C + C;
    float *part = (float *)work;
    hipLaunchKernelGGL(k_small_wgrad<0>, dim3(nc), dim3(256), 0, st, x, (const uint16_t *)nullptr,
                       dz, (const float *)nullptr, d, part, n_out);
    float *tmp = part + (int64_t)nc * n_out;
    reduce_parts(part, nc, n_out, 27 * C, dw, tmp, st);
    // bias sums live at offset 27*C of every partial row
    reduce_parts(part + 27 * C, nc, n_out, C, db, tmp, st);
    return hipret(hipGetLastError(), "tspnn_conv_in_bwd_weight");
}

tspnn_status tspnn_conv_out_fwd(const uint16_t *x, int32_t N, int32_t D0, int32_t D1, int32_t D2,
                                const float *w, const float *b, const float *res, float *out,
                                void *stream) {
    g_err.clear();
    if (!x || !w || !b || !out || !dims_ok(N, D0, D1, D2))
        return fail(TSPNN_E_INVALID, "tspnn_conv_out_fwd: bad arguments");
    Dims d{N, D0, D1, D2};
    hipLaunchKernelGGL(k_conv_out_fwd, dim3(nblk(d.vox(), 256)), dim3(256), 0,
                       (hipStream_t)stream, x, d, w, b, res, out);
    return hipret(hipGetLastError(), "tspnn_conv_out_fwd");
}

tspnn_status tspnn_conv_out_bwd(const uint16_t *x, const float *dout, int32_t N, int32_t D0,
                                int32_t D1, int32_t D2, const float *w, float *dw, float *db,
                                uint16_t *dz_in, void *work, void *stream) {
    g_err.clear();
    if (!x || !dout || !w || !dw || !db || !work || !dims_ok(N, D0, D1, D2))
        return fail(TSPNN_E_INVALID, "tspnn_conv_out_bwd: bad arguments");
    hipStream_t st = (hipStream_t)stream;
    Dims d{N, D0, D1, D2};
    const int nc = (int)(((int64_t)N * D0 * D1 + kRowsPerBlk - 1) / kRowsPerBlk);
    const int n_out = 27 * C + 1;
    float *part = (float *)work;
    hipLaunchKernelGGL(k_small_wgrad<1>, dim3(nc), dim3(256), 0, st, (const float *)nullptr, x,
                       (const uint16_t *)nullptr, dout, d, part, n_out);
    float *tmp = part + (int64_t)nc * n_out;
    reduce_parts(part, nc, n_out, 27 * C, dw, tmp, st);
    reduce_parts(part + 27 * C, nc, n_out, 1, db, tmp, st);
    if (dz_in)
        hipLaunchKernelGGL(k_conv_out_bwd_data, dim3(nblk(d.vox(), 256)), dim3(256), 0, st, x, dout,
                           d, w, dz_in);
    return hipret(hipGetLastError(), "tspnn_conv_out_bwd");
}

tspnn_status tspnn_conv_flip_weights(const uint16_t *w, uint16_t *wt, void *stream) {
    g_err.clear();
    if (!w || !wt) return fail(TSPNN_E_INVALID, "tspnn_conv_flip_weights: NULL");
    hipLaunchKernelGGL(k_flip, dim3(nblk(27 * C * C, 256)), dim3(256), 0, (hipStream_t)stream, w,
                       wt);
    return hipret(hipGetLastError(), "tspnn_conv_flip_weights");
}


size_t tspnn_vec_workspace(int32_t B, int64_t n) {
    const int64_t nc = (n + kVecChunk - 1) / kVecChunk;
    return sizeof(float) * (size_t)((nc + kRedGroups + 1) * (int64_t)B) + 64;
}

// sums[o] over the two fixed stages, then stored where active
static tspnn_status vec_reduce(int op, const float *a, const float *b, int32_t B, int64_t n,
                               float *diff, float *out, const int32_t *active, void *work,
                               hipStream_t st, const char *what) {
    const int nc = (int)((n + kVecChunk - 1) / kVecChunk);
    float *part = (float *)work;
    float *tmp = part + (int64_t)nc * B;
    float *sums = tmp + (int64_t)kRedGroups * B;
    if (op == 0)
        hipLaunchKernelGGL(k_vec_part<0>, dim3(nc, B), dim3(256), 0, st, a, b, n, diff, part);
    else
        hipLaunchKernelGGL(k_vec_part<1>, dim3(nc, B), dim3(256), 0, st, a, b, n, diff, part);
    reduce_parts(part, nc, B, B, sums, tmp, st);
    hipLaunchKernelGGL(k_store_masked, dim3(nblk(B, 256)), dim3(256), 0, st, sums, active, B,
                       out);
    return hipret(hipGetLastError(), what);
}

tspnn_status tspnn_residual(const float *y, const float *f, int32_t B, int64_t n, float *diff,
                            float *res, const int32_t *active, void *work, void *stream) {
    g_err.clear();
    if (!y || !f || !res || !work || B < 1 || B > 65535 || n < 1)
        return fail(TSPNN_E_INVALID, "tspnn_residual: bad arguments");
    return vec_reduce(0, y, f, B, n, diff, res, active, work, (hipStream_t)stream,
                      "tspnn_residual");
}

tspnn_status tspnn_dot(const float *a, const float *b, int32_t B, int64_t n, float *out,
                       void *work, void *stream) {
    g_err.clear();
    if (!a || !b || !out || !work || B < 1 || B > 65535 || n < 1)
        return fail(TSPNN_E_INVALID, "tspnn_dot: bad arguments");
    return vec_reduce(1, a, b, B, n, nullptr, out, nullptr, work, (hipStream_t)stream,
                      "tspnn_dot");
}

tspnn_status tspnn_axpy(float *x, const float *a, float alpha, int32_t B, int64_t n,
                        const int32_t *active, void *stream) {
    g_err.clear();
    if (!x || !a || B < 1 || n < 1) return fail(TSPNN_E_INVALID, "tspnn_axpy: bad arguments");
    const int64_t total = (int64_t)B * n;
    hipLaunchKernelGGL(k_axpy, dim3(nblk_strided(total)), dim3(256), 0, (hipStream_t)stream, x, a,
                       alpha, n, total, active);
    return hipret(hipGetLastError(), "tspnn_axpy");
}

tspnn_status tspnn_scale(const float *src, float alpha, int64_t n, float *dst, void *stream) {
    g_err.clear();
    if (!src || !dst || n < 1) return fail(TSPNN_E_INVALID, "tspnn_scale: bad arguments");
    hipLaunchKernelGGL(k_scale, dim3(nblk_strided(n)), dim3(256), 0, (hipStream_t)stream, src,
                       alpha, n, dst);
    return hipret(hipGetLastError(), "tspnn_scale");
}

tspnn_status tspnn_stream_copy(const float *src, float *dst, int64_t n, int32_t blocks,
                               void *stream) {
    g_err.clear();
    if (!src || !dst || n < 4 || n % 4 || ((uintptr_t)src | (uintptr_t)dst) % 16 ||
        blocks < 1 || blocks > TSPNN_STREAM_MAX_BLOCKS)
        return fail(TSPNN_E_INVALID, "tspnn_stream_copy: bad arguments");
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const f32x4 *)src, (f32x4 *)dst, n / 4);
    return hipret(hipGetLastError(), "tspnn_stream_copy");
}

tspnn_status tspnn_stream_read(const float *src, int64_t n, int32_t blocks, float *partial,
                               void *stream) {
    g_err.clear();
    if (!src || !partial || n < 4 || n % 4 || (uintptr_t)src % 16 || blocks < 1 ||
        blocks > TSPNN_STREAM_MAX_BLOCKS)
        return fail(TSPNN_E_INVALID, "tspnn_stream_read: bad arguments");
    hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const f32x4 *)src, n / 4, partial);
    return hipret(hipGetLastError(), "tspnn_stream_read");
}

}  // extern "C"
