// Attenuated emission model (TomoSphero Sec. 9.3, Eqs. 14-18) on gfx950.
//
// With s = sigma * rho and w = exp(-tau_1) * rho, where tau_1 is the
// projection of s along the sunward rays from the voxel centroids (Eq. 17's
// F_1, an ordinary explicit-ray geometry), a line of sight measures
//
//     y = sum_k w[v_k] exp(-T_k) len_k,    T_k = sum_{j <= k} s[v_j] len_j,
//
// its segments taken in order of distance from the detector (the inclusive
// cumulative sum of Eq. 18).  The ray-major store keeps every ray's segments
// in that order, so one lane walks its ray front to back with a running T:
// the same stream as the plain forward, two gathers per segment instead of
// one, and one exp.
//
// The backward (the gradient of <g, y> with respect to rho) needs, per
// segment k of ray i,
//     dy/dw[v_k] += g_i exp(-T_k) len_k
//     dy/ds[v_k] -= g_i len_k sum_{m >= k} w[v_m] exp(-T_m) len_m,
// the suffix sum being y_i minus the running prefix.  A first pass over the
// ray's segments gives y_i, a second emits both terms; lanes that hit the
// same voxel in the same step are summed before one atomic add, as in the
// atomic adjoint.  The chain rule through w and tau_1 (F_1^T) and the
// elementwise combination run as separate small kernels.
//
// Deterministic backward: the contributions are added as fixed-point
// integers instead of floats.  Each term is rounded to an integer multiple
// of 2^qe; the terms of a step's lanes that share a voxel are summed in LDS
// (merge_step) and the sum goes to the voxel's signed 64-bit accumulator
// with one integer atomic add.  Integer addition is exact and associative,
// so the sums (and the float each voxel finally gets) do not depend on the
// order in which the adds land: bitwise reproducible.  qe comes from a bound
// on every voxel's sum of |terms| (fixed_exponent), which keeps every
// partial sum below 2^62 quanta; each term's rounding is at most 2^(qe-1).

#include "tsp_internal.h"

namespace tsp {
namespace {

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

typedef float v4f __attribute__((ext_vector_type(4)));

// s[b][v] = sigma[v] * rho[b][v]
__global__ void k_atten_s(const float *sigma, const float *rho, int64_t V, int64_t n, float *s) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) s[i] = sigma[i % V] * rho[i];
}

// w = exp(-tau1) * rho
__global__ void k_atten_w(const float *tau1, const float *rho, int64_t n, float *w) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) w[i] = expf(-tau1[i]) * rho[i];
}

// out = -w * gw  (gradient reaching tau_1)
__global__ void k_atten_gtau(const float *w, const float *gw, int64_t n, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) out[i] = -w[i] * gw[i];
}

// grad = exp(-tau1) * gw + sigma * (gs + gs_sun)
__global__ void k_atten_grad(const float *tau1, const float *sigma, const float *gw,
                             const float *gs, const float *gs_sun, int64_t V, int64_t n,
                             float *grad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        grad[i] = expf(-tau1[i]) * gw[i] + sigma[i % V] * (gs[i] + gs_sun[i]);
}

// One lane per ray slot of the ray-major store (see tsp_apply.hip for the
// layout); entry j of the lane at sell_index(base, lane, j), j in order of
// distance from the detector, voxels rebuilt from the entry codes; escape
// and padding entries carry no length.
__global__ __launch_bounds__(256) void k_fwd_atten(const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ cnt_sorted,
                                                    const int64_t *__restrict__ slice_ptr,
                                                    const int32_t *__restrict__ slice_len,
                                                    const uint8_t *__restrict__ code,
                                                    const float *__restrict__ len,
                                                    int64_t n_slots, const float *__restrict__ s,
                                                    const float *__restrict__ w, int na, int nena,
                                                    float *__restrict__ y) {
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;
    const int32_t ray = perm[slot];
    if (ray < 0) return;
    const int c = cnt_sorted[slot];
    const int64_t base = slice_ptr[slot >> 6];
    const int lane = (int)(slot & 63);
    const uint32_t *cp = (const uint32_t *)(code + base) + lane;
    const v4f *lp = (const v4f *)(len + base) + lane;
    float T = 0.0f, acc = 0.0f;
    int32_t v = 0;
    for (int q = 0; q < ((c + 3) >> 2); q++) {
        const uint32_t cw = __builtin_nontemporal_load(cp + (int64_t)q * kWave);
        const v4f lq = __builtin_nontemporal_load(lp + (int64_t)q * kWave);
        const float la[4] = {lq[0], lq[1], lq[2], lq[3]};
        // escapes and the padding past the ray's last entry carry length 0,
        // which leaves T and the sum as they are: no branch per entry
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int cd = (cw >> (8 * e)) & 255;
            const float l = decode_entry(cd, la[e], v, na, nena);
            T = fmaf(s[v], l, T);
            acc = fmaf(w[v] * expf(-T), l, acc);
        }
    }
    y[ray] = acc;
}

// Add v into the 64-bit fixed-point accumulator acc[i]: v rounded to an
// integer multiple of 2^qe (nearest, ties to even; the scaling by a power
// of two is exact).
__device__ __forceinline__ void fixed_add(unsigned long long *acc, int64_t i, float v, int qe) {
    const long long q = (long long)rint(ldexp((double)v, -qe));
    if (q != 0) atomicAdd(acc + i, (unsigned long long)q);
}

// Scale exponent of the fixed-point sums.  Every line of sight adds to a
// voxel at most max|g| len (the w-gradient: exp(-T) <= 1) and max|g| len
// 2R max|w| (the s-gradient: a suffix sum stays below the outer sphere's
// diameter 2R times max|w|), and its lengths add up to at most 2R, so
// M = 2 max|g| nrays 2R (1 + 2R max|w|) bounds twice any voxel's sum of
// |terms| (the factor 2 covers the float rounding of merged terms and
// lengths); q = ilogb(M) + 1 - 62 keeps every partial sum below 2^62 quanta.
// bits[0], bits[1] hold max|g| and max|w| as float bits (non-negative
// floats order like their bit patterns).
__device__ __forceinline__ int fixed_exponent(const unsigned *bits, double two_r, double nrays) {
    const double mg = (double)__uint_as_float(bits[0]);
    const double mw = (double)__uint_as_float(bits[1]);
    const double M = 2.0 * fmax(mg, 1e-30) * nrays * two_r * (1.0 + two_r * mw);
    return ilogb(M) + 1 - 62;
}

// out[0] = max |a| over n floats, as float bits, by atomicMax (out zeroed first)
__global__ void k_absmax(const float *__restrict__ a, int64_t n, unsigned *out) {
    unsigned m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(fabsf(a[i])));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, m);
}

// x[i] = the fixed-point sum acc[i] times 2^qe, converted once (through
// double) to float.
__global__ void k_fixed_to_float(const unsigned long long *acc, int64_t V,
                                 const unsigned *bits, double two_r, double nrays, float *x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    x[i] = (float)ldexp((double)(long long)acc[i], fixed_exponent(bits, two_r, nrays));
}

// One step of the backward's scatter: the lanes of a wavefront that hold
// the same voxel add their two terms in LDS and one lane per voxel adds the
// sums to the voxel's gradients.  Each active lane writes its lane id into a
// slot of a per-wavefront table chosen by a hash of its voxel, then reads the
// slot back: the lane found there (the last writer) owns the voxel when it
// holds the same voxel, and the lanes of the voxel add into the owner's pair
// of accumulators; a lane whose slot went to another voxel adds directly.
// The owners then take their sums (and reset them) and add them globally.
// LDS operations of one wavefront execute in order, so each phase sees the
// previous one; the fences keep the compiler from reordering the phases.
// FIXED: terms are rounded to multiples of 2^qe one by one and summed as
// 64-bit integers (order-independent); else float LDS adds and atomics.
constexpr int kMergeSlots = 256;
template <bool FIXED, class Acc>
__device__ __forceinline__ void merge_step(int v, float a, float bterm, int lane, int *tb,
                                           Acc *sa, Acc *sb, float *gw, float *gs,
                                           unsigned long long *acc, int64_t V, int qe) {
    const bool act = v >= 0;
    const int h = (int)(((unsigned)v * 2654435761u) >> 24);  // 8 bits: kMergeSlots
    if (act) __hip_atomic_store(tb + h, lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    const int owner = act ? __hip_atomic_load(tb + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT)
                          : lane;
    const int ov = __shfl(v, owner, kWave);
    Acc ta, tbv;
    if (FIXED) {
        ta = (Acc)(long long)rint(ldexp((double)a, -qe));
        tbv = (Acc)(long long)rint(ldexp((double)bterm, -qe));
    } else {
        ta = (Acc)a;
        tbv = (Acc)bterm;
    }
    if (act && ov == v) {
        atomicAdd(sa + owner, ta);
        atomicAdd(sb + owner, tbv);
    } else if (act) {  // the slot went to another voxel
        if (FIXED) {
            if (ta) atomicAdd(acc + v, (unsigned long long)ta);
            if (tbv) atomicAdd(acc + V + v, (unsigned long long)tbv);
        } else {
            atomicAdd(gw + v, (float)ta);
            atomicAdd(gs + v, (float)tbv);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (act && owner == lane) {
        const Acc xa = atomicExch(sa + lane, (Acc)0), xb = atomicExch(sb + lane, (Acc)0);
        if (FIXED) {
            if (xa) atomicAdd(acc + v, (unsigned long long)xa);
            if (xb) atomicAdd(acc + V + v, (unsigned long long)xb);
        } else {
            atomicAdd(gw + v, (float)xa);
            atomicAdd(gs + v, (float)xb);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <bool FIXED>
__global__ __launch_bounds__(256) void k_bwd_atten(const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ cnt_sorted,
                                                    const int64_t *__restrict__ slice_ptr,
                                                    const int32_t *__restrict__ slice_len,
                                                    const uint8_t *__restrict__ code,
                                                    const float *__restrict__ len,
                                                    int64_t n_slots, const float *__restrict__ s,
                                                    const float *__restrict__ w,
                                                    const float *__restrict__ gy, int na,
                                                    int nena, float *gw, float *gs,
                                                    unsigned long long *acc, int64_t V,
                                                    const unsigned *bits, double two_r,
                                                    double nrays) {
    // FIXED: acc holds the fixed-point sums of gw ([V]) then of gs ([V])
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;  // n_slots is a multiple of 256: whole wavefronts
    const int qe = FIXED ? fixed_exponent(bits, two_r, nrays) : 0;
    const int lane = (int)(slot & 63);
    const int32_t ray = perm[slot];
    const int c = (ray >= 0) ? cnt_sorted[slot] : 0;
    const int m = slice_len[slot >> 6];
    const int64_t base = slice_ptr[slot >> 6];
    const float g = (ray >= 0) ? gy[ray] : 0.0f;
    // per wavefront: the voxel table and one pair of accumulators per lane
    using Acc = typename std::conditional<FIXED, unsigned long long, float>::type;
    __shared__ int tbl[4][kMergeSlots];
    __shared__ Acc accs[4][2][kWave];
    const int wv = threadIdx.x >> 6;
    int *tb = tbl[wv];
    Acc *sa = accs[wv][0], *sb = accs[wv][1];
    sa[lane] = (Acc)0;
    sb[lane] = (Acc)0;
    // pass 1: the ray's measurement (the total that the suffix sums start from)
    const uint32_t *cp = (const uint32_t *)(code + base) + lane;
    const v4f *lp = (const v4f *)(len + base) + lane;
    float T = 0.0f, yr = 0.0f;
    int32_t vr = 0;
    for (int q = 0; q < ((c + 3) >> 2); q++) {
        const uint32_t cw = cp[(int64_t)q * kWave];
        const v4f lq = lp[(int64_t)q * kWave];
        const float la[4] = {lq[0], lq[1], lq[2], lq[3]};
#pragma unroll
        for (int e = 0; e < 4; e++) {  // escapes and padding: length 0, no change
            const int cd = (cw >> (8 * e)) & 255;
            const float l = decode_entry(cd, la[e], vr, na, nena);
            T = fmaf(s[vr], l, T);
            yr = fmaf(w[vr] * expf(-T), l, yr);
        }
    }
    // pass 2: both gradient terms of every segment, merged across the wavefront
    T = 0.0f;
    float prefix = 0.0f;
    vr = 0;
    for (int q = 0; q < (m >> 2); q++) {  // m is uniform over the wavefront, a multiple of 4
        const uint32_t cw = cp[(int64_t)q * kWave];
        const v4f lq = lp[(int64_t)q * kWave];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            // escapes and padding carry length 0: T, the prefix and both
            // terms stay as they are, with no branch per entry
            const int cd = (cw >> (8 * e)) & 255;
            const float l = decode_entry(cd, lq[e], vr, na, nena);
            const int v = (4 * q + e < c && cd != kCodeEsc) ? vr : -1;
            T = fmaf(s[vr], l, T);
            const float E = expf(-T);
            const float ck = w[vr] * E * l;
            const float a = g * E * l;
            const float bterm = -g * l * (yr - prefix);
            prefix += ck;
            if (FIXED) {
                merge_step<FIXED>(v, a, bterm, lane, tb, sa, sb, gw, gs, acc, V, qe);
            } else {
                // the float path merges by leaders (one wavefront sum per
                // distinct voxel, at most kMaxMerges): float LDS adds under
                // the table merge ran 3.7 ms against 2.6 ms at Medium
                uint64_t pend = __ballot(v >= 0);  // uniform: every lane is active
                for (int it = 0; pend && it < kMaxMerges; it++) {
                    const int leader = __ffsll((unsigned long long)pend) - 1;
                    const int v0 = __builtin_amdgcn_readlane(v, leader);
                    const bool mine = (v == v0);
                    const float sa0 = wave_sum_f32(mine ? a : 0.0f);
                    const float sb0 = wave_sum_f32(mine ? bterm : 0.0f);
                    if (lane == leader) {
                        atomicAdd(gw + v0, sa0);
                        atomicAdd(gs + v0, sb0);
                    }
                    pend &= ~__ballot(mine);
                }
                if ((pend >> lane) & 1ull) {  // past the merge limit
                    atomicAdd(gw + v, a);
                    atomicAdd(gs + v, bterm);
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_absmax(const float *a, int64_t n, unsigned *out, hipStream_t st) {
    hipLaunchKernelGGL(k_absmax, dim3(256), dim3(256), 0, st, a, n, out);
    return hipGetLastError();
}

hipError_t launch_atten_s(const float *sigma, const float *rho, int64_t V, int B, float *s,
                          hipStream_t st) {
    const int64_t n = V * B;
    hipLaunchKernelGGL(k_atten_s, dim3(strided_blocks(n)), dim3(256), 0, st, sigma, rho, V, n,
                       s);
    return hipGetLastError();
}

hipError_t launch_atten_w(const float *tau1, const float *rho, int64_t n, float *w,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_atten_w, dim3(strided_blocks(n)), dim3(256), 0, st, tau1, rho, n, w);
    return hipGetLastError();
}

hipError_t launch_atten_gtau(const float *w, const float *gw, int64_t n, float *out,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_atten_gtau, dim3(strided_blocks(n)), dim3(256), 0, st, w, gw, n, out);
    return hipGetLastError();
}

hipError_t launch_atten_grad(const float *tau1, const float *sigma, const float *gw,
                             const float *gs, const float *gs_sun, int64_t V, int B, float *grad,
                             hipStream_t st) {
    const int64_t n = V * B;
    hipLaunchKernelGGL(k_atten_grad, dim3(strided_blocks(n)), dim3(256), 0, st, tau1, sigma, gw,
                       gs, gs_sun, V, n, grad);
    return hipGetLastError();
}

hipError_t launch_fwd_atten(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                            const int64_t *slice_ptr, const int32_t *slice_len,
                            const uint8_t *code, const float *len, const float *s, const float *w,
                            int B, int64_t V, int na, int nena, float *y, hipStream_t st) {
    for (int b = 0; b < B; b++) {
        hipLaunchKernelGGL(k_fwd_atten, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, perm,
                           cnt_sorted, slice_ptr, slice_len, code, len, rd.n_slots, s + b * V,
                           w + b * V, na, nena, y + b * rd.R);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_bwd_atten(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                            const int64_t *slice_ptr, const int32_t *slice_len,
                            const uint8_t *code, const float *len, const float *s, const float *w,
                            const float *gy, int B, int64_t V, int na, int nena, double r_out,
                            float *gw, float *gs, void *ws, hipStream_t st) {
    const double two_r = 2.0 * r_out, nrays = (double)rd.R;
    for (int b = 0; b < B; b++) {
        const unsigned grid = blocks_for(rd.n_slots, 256);
        if (!ws) {
            hipLaunchKernelGGL(k_bwd_atten<false>, dim3(grid), dim3(256), 0, st, perm, cnt_sorted,
                               slice_ptr, slice_len, code, len, rd.n_slots, s + b * V, w + b * V,
                               gy + b * rd.R, na, nena, gw + b * V, gs + b * V, nullptr, V,
                               nullptr, two_r, nrays);
        } else {
            unsigned long long *acc = (unsigned long long *)ws;
            unsigned *bits = (unsigned *)(acc + 2 * V);
            // cleared by a kernel (not a memset node, should a caller capture this)
            hipError_t e = launch_zero_u64(acc, 2 * V + 1, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_absmax, dim3(256), dim3(256), 0, st, gy + b * rd.R, rd.R, bits);
            hipLaunchKernelGGL(k_absmax, dim3(256), dim3(256), 0, st, w + b * V, V, bits + 1);
            hipLaunchKernelGGL(k_bwd_atten<true>, dim3(grid), dim3(256), 0, st, perm, cnt_sorted,
                               slice_ptr, slice_len, code, len, rd.n_slots, s + b * V, w + b * V,
                               gy + b * rd.R, na, nena, nullptr, nullptr, acc, V, bits, two_r,
                               nrays);
            hipLaunchKernelGGL(k_fixed_to_float, dim3(blocks_for(V, 256)), dim3(256), 0, st, acc,
                               V, bits, two_r, nrays, gw + b * V);
            hipLaunchKernelGGL(k_fixed_to_float, dim3(blocks_for(V, 256)), dim3(256), 0, st,
                               acc + V, V, bits, two_r, nrays, gs + b * V);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t atten_fixed_ws_bytes(int64_t V) { return (size_t)V * 16 + 64; }

}  // namespace tsp
