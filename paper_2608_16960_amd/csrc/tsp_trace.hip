// Ray tracing through a spherical grid on gfx950: steps 1-3 of TomoSphero
// (Sec. 3.1 intersections, Sec. 3.2 crossing directions, Sec. 3.3 ordering
// and lengths) fused per ray, plus the on-the-fly forward / adjoint that feed
// every segment straight into step 4 (Sec. 3.4, Eq. 5).
//
// One ray per lane.  Instead of materialising the padded crossing arrays of
// Sec. 3.1 and sorting them (Sec. 3.3), each lane walks three crossing
// streams that are already ordered by distance:
//   radial      spheres r_b[k]: inbound roots in decreasing k, then outbound
//               roots in increasing k; every inbound crossing is "negative"
//               and every outbound one "positive" (Eq. 11), so the region
//               index becomes k-1 or k;
//   elevation   cones cos(theta) = cos(e_b[k]); along a line the colatitude
//               has at most one turning point, at the distance where Eq. 12's
//               m.n vanishes, so the crossings form at most two monotone runs;
//               the regions at the run ends fix which cones are crossed, and
//               Eq. 12's sign at each root picks the root of the cone's
//               quadratic that belongs to the run;
//   azimuth     half-planes a_b[k]: the azimuth is monotone along a line, in
//               the direction of (p x n)_z (Eq. 13), sweeping less than pi.
// The lane merges the three streams by distance (ties: radial, elevation,
// azimuth), updates one index per crossing as in Table 2(b), skips rows with
// an invalid index (Table 2(c)), and merges touching pieces of the same voxel
// into one canonical segment.
//
// The lane classifies the ray's entry point on the outermost sphere (the
// region of the start point of Table 2(a), advanced past the crossings that
// lie outside the grid, which cannot contribute).
//
// All geometry is FP64; boundary tables are staged in LDS.  The file is
// compiled with -ffp-contract=off so that the counting and the filling
// kernels, which re-trace the same ray, evaluate identical arithmetic.

#include <cmath>
#include <type_traits>

#include "tsp_internal.h"
#include "tsp_trace_core.h"

namespace tsp {
namespace {

using namespace core;

__device__ __forceinline__ void ray_of(const RayDesc &rd, int32_t ray, V3 &x, V3 &n) {
    if (rd.explicit_rays) {
        const double *s = rd.starts + 3 * (int64_t)ray;
        const double *d = rd.dirs + 3 * (int64_t)ray;
        x = {s[0], s[1], s[2]};
        n = {d[0], d[1], d[2]};
        return;
    }
    const int hw = rd.H * rd.W;
    const int view = ray / hw;
    const int rem = ray - view * hw;
    const int i = rem / rd.W, j = rem - (rem / rd.W) * rd.W;
    const double *f = rd.frames + 16 * view;
    const double sy = (2.0 * (i + 0.5) / rd.H - 1.0) * f[12];
    const double sx = (2.0 * (j + 0.5) / rd.W - 1.0) * f[13];
    if (f[14] != 0.0) {  // parallel beam: pixel centre on the detector plane, along w
        x = {f[0] + sx * f[6] + sy * f[9], f[1] + sx * f[7] + sy * f[10],
             f[2] + sx * f[8] + sy * f[11]};
        n = {f[3], f[4], f[5]};
        return;
    }
    double d0 = f[3] + sx * f[6] + sy * f[9];
    double d1 = f[4] + sx * f[7] + sy * f[10];
    double d2 = f[5] + sx * f[8] + sy * f[11];
    const double dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    x = {f[0], f[1], f[2]};
    n = {d0 / dn, d1 / dn, d2 / dn};
}

// ---------------------------------------------------------------- visitors

// Entries of the ray-major store (codec in tsp_internal.h): one per segment,
// two where the voxel does not follow from the previous one by a coded step
// (always for the first segment).
struct CountVis {
    int n = 0;     // store entries
    int segs = 0;  // canonical segments
    int32_t prev = -1;
    int na, nena;
    __device__ void seg(int v, double) {
        n += (prev < 0 || step_code(v - prev, na, nena) == kCodeEsc) ? 2 : 1;
        prev = v;
        segs++;
    }
};

struct FillVis {
    uint8_t *code;
    float *len;
    int64_t base;
    int lane;
    int cap;
    int na, nena;
    int n = 0;
    int32_t prev = -1;
    __device__ void put(int c, float l) {
        if (n < cap) {
            const int64_t i = sell_index(base, lane, n);
            code[i] = (uint8_t)c;
            len[i] = l;
        }
        n++;
    }
    __device__ void seg(int v, double l) {
        int c = (prev < 0) ? kCodeEsc : step_code(v - prev, na, nena);
        if (c == kCodeEsc) {
            put(kCodeEsc, __int_as_float(v));
            c = 0;
        }
        put(c, (float)l);
        prev = v;
    }
};

// NB == 1: rho is [V]; NB == 4: rho is voxel-major [V][4] (one 16-byte gather
// per segment serves the whole batch).
template <int NB>
struct FwdVis {
    const float *rho;
    float acc[NB];
    __device__ void seg(int v, double l) {
        const float lf = (float)l;
        if (NB == 1) {
            acc[0] = fmaf(lf, rho[v], acc[0]);
        } else {
            const float4 r = reinterpret_cast<const float4 *>(rho)[v];
            acc[0] = fmaf(lf, r.x, acc[0]);
            acc[1] = fmaf(lf, r.y, acc[1]);
            acc[2] = fmaf(lf, r.z, acc[2]);
            acc[3] = fmaf(lf, r.w, acc[3]);
        }
    }
};

// Workgroups are dispatched to the 8 XCDs round-robin; this remaps block b so
// that each XCD walks a contiguous run of windows (consecutive windows cover
// a compact detector patch, whose rays share voxels in that XCD's L2).
__device__ __forceinline__ int64_t xcd_window(int64_t nwin) {
    const int64_t per = gridDim.x / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// ---------------------------------------------------------------- kernels

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// Per natural slot: store entries (cnt_nat) and canonical segments (seg_nat,
// may be null); total and maxcnt over segments; per window (a workgroup's
// 256 slots) the canonical segments, added into win_seg (zeroed first; may
// be null).
__global__ __launch_bounds__(256) void k_count(TabDesc D, const double *tab, RayDesc rd,
                                                int32_t *cnt_nat, int32_t *seg_nat,
                                                unsigned long long *total, int *maxcnt,
                                                int32_t *win_seg) {
    extern __shared__ double lds[];
    stage_tables(D, tab, lds);
    const Tab T = make_tab(D, lds);
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int c = 0;
    if (slot < rd.n_slots) {
        const int32_t ray = natural_ray(rd, slot);
        int e = 0;
        if (ray >= 0) {
            V3 x, n;
            ray_of(rd, ray, x, n);
            CountVis vis;
            vis.na = D.na;
            vis.nena = D.ne * D.na;
            trace_ray(T, x, n, vis);
            c = vis.segs;
            e = vis.n;
        }
        if (cnt_nat) cnt_nat[slot] = e;
        if (seg_nat) seg_nat[slot] = c;
    }
    const int s = wave_sum_i(c);
    const int m = wave_max_i(c);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(total, (unsigned long long)s);
        atomicMax(maxcnt, m);
        if (win_seg) atomicAdd(win_seg + blockIdx.x, s);
    }
}

__global__ __launch_bounds__(256) void k_fill(TabDesc D, const double *tab, RayDesc rd,
                                               const int32_t *perm, const int32_t *cnt_sorted,
                                               const int64_t *slice_ptr,
                                               const int32_t *slice_len, uint8_t *code,
                                               float *len, int *err) {
    extern __shared__ double lds[];
    stage_tables(D, tab, lds);
    const Tab T = make_tab(D, lds);
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= rd.n_slots) return;
    const int64_t s = slot / kWave;
    const int lane = (int)(slot % kWave);
    const int32_t ray = perm[slot];
    const int cap = cnt_sorted[slot];
    const int m = slice_len[s];
    const int64_t base = slice_ptr[s];
    int n = 0;
    if (ray >= 0) {
        V3 x, nn;
        ray_of(rd, ray, x, nn);
        FillVis vis{code, len, base, lane, cap, D.na, D.ne * D.na};
        trace_ray(T, x, nn, vis);
        n = vis.n;
        if (n != cap) atomicOr(err, 1);
    }
    for (int j = min(n, cap); j < m; j++) {  // padding up to the slice length
        const int64_t i = sell_index(base, lane, j);
        code[i] = 0;
        len[i] = 0.0f;
    }
}

template <int NB>
__global__ __launch_bounds__(256) void k_otf_forward(TabDesc D, const double *tab, RayDesc rd,
                                                      const float *rho, int nb, int64_t V,
                                                      float *y) {
    extern __shared__ double lds[];
    stage_tables(D, tab, lds);
    const Tab T = make_tab(D, lds);
    const int64_t win = xcd_window(rd.n_slots / kWindow);
    if (win >= rd.n_slots / kWindow) return;  // padding blocks of the remapped grid
    const int64_t slot = win * kWindow + threadIdx.x;
    const int32_t ray = natural_ray(rd, slot);
    if (ray < 0) return;
    V3 x, n;
    ray_of(rd, ray, x, n);
    FwdVis<NB> vis;
    vis.rho = rho + NB * frame_base(rd.obj_frame, (int64_t)rd.H * rd.W, ray,
                                    (int64_t)D.nr * D.ne * D.na);
#pragma unroll
    for (int b = 0; b < NB; b++) vis.acc[b] = 0.0f;
    trace_ray(T, x, n, vis);
#pragma unroll
    for (int b = 0; b < NB; b++)
        if (b < nb) y[b * rd.R + ray] = vis.acc[b];
}

// Value of lane l + K in lane l (row_shl:K within rows of 16; 0 past the row).
template <int K>
__device__ __forceinline__ float dpp_from_up(float x) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x100 + K, 0xf, 0xf, false));
}
template <int K>
__device__ __forceinline__ long long dpp_from_up(long long x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(x & 0xffffffffll), 0x100 + K, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), 0x100 + K, 0xf, 0xf, false);
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Lanes l and l + K (bit K of l clear, K <= 8: both in one row of 16) that
// hold the same voxel (v >= 0) add their values in lane l; lane l + K drops
// out (v = -1).  Every lane of the wavefront must be active.
template <int K, int NB, class T>
__device__ __forceinline__ void merge_pairs(int &v, T *val, int lane) {
    const int up = __builtin_amdgcn_update_dpp(-1, v, 0x100 + K, 0xf, 0xf, false);  // row_shl:K
    const int dn = __builtin_amdgcn_update_dpp(-1, v, 0x110 + K, 0xf, 0xf, false);  // row_shr:K
    const bool low = (lane & K) == 0;
    const bool take = low && v >= 0 && up == v;
    const bool give = !low && v >= 0 && dn == v;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const T t = dpp_from_up<K>(val[b]);
        if (take) val[b] += t;
    }
    if (give) v = -1;
}

// On-the-fly adjoint into x ([V] for one object, voxel-major [V][4] for a
// batch).  The 256 rays of a window cross largely the same voxels, so the
// workgroup first adds its contributions in a hash table in LDS (open
// addressing on the voxel index, native LDS float adds, values stored object
// by object so that the lanes of one add spread over the banks) and only a
// flush issues global atomics, one per distinct voxel and object.  The rays
// advance kOtfEvents boundary events between workgroup barriers; at a barrier
// the table is flushed once it is more than half full, and after the last ray
// ends.  Before inserting, the lanes of neighbouring rays that reached the
// same voxel in the same event add their values in registers (pairs at lane
// distance 1, 2, 4, 8 through DPP row shifts), which removes about half of
// the LDS atomics and most of their same-address serialisation; a slot is
// claimed (or found taken) by one compare-and-swap per probe, and the adds
// follow the probe loop.  An insertion that finds no slot within kOtfProbes
// probes goes straight to a global atomic, so a crowded table costs speed,
// never correctness.
constexpr int kOtfEvents = 16;
constexpr int kOtfProbes = 8;
// FIX: values are 64-bit fixed-point integers (the reproducible variant below)
template <int NB, bool FIX = false> struct OtfHash {
    using Val = typename std::conditional<FIX, long long, float>::type;
    static constexpr int kSize = FIX ? 1024 : (NB == 1 ? 2048 : 1024);  // power of two
    static constexpr size_t kBytes = (size_t)kSize * (4 + NB * sizeof(Val));
    static_assert(kBytes <= kOtfHashBytes, "hash table exceeds its LDS reserve");
};

// Reproducible sums in fixed point.  Object b's terms len * y are rounded to
// integer multiples of 2^q_b (round to nearest even) and added as 64-bit
// integers, so that every order of addition gives the same sum.  q_b follows
// from M_b = max |y_b| * lsum, lsum = 2 * (rays) * (diameter of the outer
// sphere) >= twice the summed lengths of all rays, which bounds every voxel's
// sum of |terms|: q_b = ilogb(M_b) + 1 - 62 keeps it, and so every partial
// sum, below 2^62 quanta.
__device__ __forceinline__ int fix_exponent(unsigned ybits, double lsum) {
    return ilogb(fmax((double)__uint_as_float(ybits), 1e-30) * lsum) + 1 - 62;
}

// The batch-4 kernel allocates 96 VGPRs, five wavefronts per SIMD, with the
// measurements in LDS (99 and four wavefronts with them in registers, about
// 3% slower; asking for five with amdgpu_waves_per_eu spills instead).
__device__ __forceinline__ void lds_add(float *p, float v) { atomicAdd(p, v); }
__device__ __forceinline__ void lds_add(long long *p, long long v) {
    atomicAdd(reinterpret_cast<unsigned long long *>(p), (unsigned long long)v);
}
__device__ __forceinline__ void global_add(float *x, unsigned long long *, int64_t i, float v) {
    atomicAdd(x + i, v);
}
__device__ __forceinline__ void global_add(float *, unsigned long long *acc, int64_t i,
                                           long long v) {
    atomicAdd(acc + i, (unsigned long long)v);
}

// FIX: the sums go in 64-bit fixed point (fix_exponent) into acc_out (same
// layout as x_out) instead of float atomics into x_out; ybits[b] holds
// max |y| of object b as float bits.
template <int NB, bool FIX>
__global__ __launch_bounds__(256) void k_otf_adjoint(TabDesc D, const double *tab, RayDesc rd,
                                                      const float *y, int nb, int64_t V,
                                                      float *x_out, unsigned long long *acc_out,
                                                      const unsigned *ybits, double lsum) {
    using Val = typename OtfHash<NB, FIX>::Val;
    constexpr int HS = OtfHash<NB, FIX>::kSize;
    extern __shared__ double lds[];  // grid tables, hash keys and values, measurements
    __shared__ int fill;
    stage_tables(D, tab, lds);
    const Tab T = make_tab(D, lds);
    int *hkey = reinterpret_cast<int *>(lds + D.n_tab);
    Val *hval = reinterpret_cast<Val *>(hkey + HS);  // [NB][HS]
    const int64_t win = xcd_window(rd.n_slots / kWindow);
    if (win >= rd.n_slots / kWindow) return;  // whole padding blocks of the remapped grid
    for (int i = threadIdx.x; i < HS; i += 256) {
        hkey[i] = -1;
#pragma unroll
        for (int b = 0; b < NB; b++) hval[b * HS + i] = (Val)0;
    }
    if (threadIdx.x == 0) fill = 0;
    const int64_t slot = win * kWindow + threadIdx.x;
    const int32_t ray = natural_ray(rd, slot);
    float yv[NB];
    double sc[NB];  // FIX: 2^-q_b
    bool any = false;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        yv[b] = (ray >= 0 && b < nb) ? y[b * rd.R + ray] : 0.0f;
        any |= (yv[b] != 0.0f);
        sc[b] = FIX ? ldexp(1.0, -fix_exponent(ybits[b < nb ? b : 0], lsum)) : 1.0;
    }
    // the ray's measurements wait in LDS, read back at every event, rather
    // than in registers: four fewer VGPRs hold the batch-4 kernel at 96,
    // five wavefronts per SIMD instead of four
    float *ysh = reinterpret_cast<float *>(hval + NB * HS) + threadIdx.x * NB;
#pragma unroll
    for (int b = 0; b < NB; b++) ysh[b] = yv[b];
    Walker w;
    bool alive = false;
    int32_t fb = 0;  // object frame of this ray, in voxels
    if (ray >= 0 && any) {  // a zero measurement contributes nothing
        V3 x, n;
        ray_of(rd, ray, x, n);
        alive = w.init(T, x, n);
        fb = (int32_t)frame_base(rd.obj_frame, (int64_t)rd.H * rd.W, ray,
                                 (int64_t)D.nr * D.ne * D.na);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    for (;;) {
        for (int k = 0; k < kOtfEvents; k++) {
            if (__ballot(alive) == 0) break;  // uniform over the wavefront
            int v = -1;
            float lf = 0.0f;
            if (alive) {
                int vv;
                double l;
                const bool seg = w.step(T, vv, l);
                alive = !w.done();
                if (seg) {
                    v = vv + fb;
                    lf = (float)l;
                }
            }
            Val val[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) {
                if (FIX)  // the product of two floats is exact in double
                    val[b] = (Val)rint((double)lf * (double)ysh[b] * sc[b]);
                else
                    val[b] = (Val)(lf * ysh[b]);
            }
            merge_pairs<1, NB>(v, val, lane);
            merge_pairs<2, NB>(v, val, lane);
            merge_pairs<4, NB>(v, val, lane);
            merge_pairs<8, NB>(v, val, lane);
            bool claimed = false;
            int hs = -1;  // the voxel's table slot, once found
            if (v >= 0) {
                unsigned h = ((unsigned)v * 2654435761u) >> (32 - __builtin_ctz(HS));
                for (int p = 0; p < kOtfProbes; p++) {
                    // claim an empty slot, or learn whose it is
                    const int key = atomicCAS(hkey + h, -1, v);
                    claimed = key == -1;
                    if (key == -1 || key == v) {
                        hs = (int)h;
                        break;
                    }
                    h = (h + 1) & (HS - 1);
                }
            }
            // the adds after the probe loop: one set of LDS adds per
            // wavefront step, whatever the lanes' probe counts
            if (hs >= 0) {
#pragma unroll
                for (int b = 0; b < NB; b++) lds_add(hval + b * HS + hs, val[b]);
            } else if (v >= 0) {
#pragma unroll
                for (int b = 0; b < NB; b++)
                    if (b < nb) global_add(x_out, acc_out, (int64_t)v * NB + b, val[b]);
            }
            // one add to the fill count per wavefront, not one per claim on a
            // single LDS word (every lane is active here)
            const uint64_t cl = __ballot(claimed);
            if (lane == 0 && cl) atomicAdd(&fill, (int)__popcll(cl));
        }
        __syncthreads();  // every insertion of this round has landed
        const int f = fill;
        const bool more = __syncthreads_or(alive);  // also: every thread has read fill
        if (f > HS / 2 || !more) {
            for (int i = threadIdx.x; i < HS; i += 256) {
                const int key = hkey[i];
                if (key < 0) continue;
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    if (b < nb) global_add(x_out, acc_out, (int64_t)key * NB + b, hval[b * HS + i]);
                    hval[b * HS + i] = (Val)0;
                }
                hkey[i] = -1;
            }
            if (threadIdx.x == 0) fill = 0;
            __syncthreads();
        }
        if (!more) break;
    }
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) p[i] = 0ull;
}

// x[b][v] = the fixed-point sum acc[v * NB + b] times 2^q_b, rounded to float
// (through double); b < nb.
__global__ void k_fix_to_float(const unsigned long long *acc, int NB, int nb, int64_t V,
                               const unsigned *ybits, double lsum, float *x) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nb * V;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i / V);
        const int64_t v = i - (int64_t)b * V;
        const long long a = (long long)acc[v * NB + b];
        x[i] = (float)ldexp((double)a, fix_exponent(ybits[b], lsum));
    }
}

__global__ void k_rays(RayDesc rd, double *starts, double *dirs) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rd.R) return;
    V3 x, n;
    ray_of(rd, (int32_t)r, x, n);
    if (starts) {
        starts[3 * r + 0] = x.x;
        starts[3 * r + 1] = x.y;
        starts[3 * r + 2] = x.z;
    }
    if (dirs) {
        dirs[3 * r + 0] = n.x;
        dirs[3 * r + 1] = n.y;
        dirs[3 * r + 2] = n.z;
    }
}

inline unsigned grid_of(int64_t n_slots) { return (unsigned)((n_slots + 255) / 256); }

}  // namespace

hipError_t launch_count(const TabDesc &T, const double *tab, const RayDesc &rd, int32_t *cnt_nat,
                        int32_t *seg_nat, unsigned long long *total, int *maxcnt,
                        int32_t *win_seg, hipStream_t st) {
    hipLaunchKernelGGL(k_count, dim3(grid_of(rd.n_slots)), dim3(256), T.n_tab * sizeof(double),
                       st, T, tab, rd, cnt_nat, seg_nat, total, maxcnt, win_seg);
    return hipGetLastError();
}

hipError_t launch_fill(const TabDesc &T, const double *tab, const RayDesc &rd,
                       const int32_t *perm, const int32_t *cnt_sorted, const int64_t *slice_ptr,
                       const int32_t *slice_len, uint8_t *code, float *len, int *err,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_fill, dim3(grid_of(rd.n_slots)), dim3(256), T.n_tab * sizeof(double), st,
                       T, tab, rd, perm, cnt_sorted, slice_ptr, slice_len, code, len, err);
    return hipGetLastError();
}

// [B][V] <-> voxel-major [V][4] for batch chunks of up to 4 objects
__global__ void k_to_vmajor(const float *src, int nb, int64_t V, float *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V * 4;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(i & 3);
        dst[i] = (b < nb) ? src[(int64_t)b * V + (i >> 2)] : 0.0f;
    }
}

__global__ void k_from_vmajor(const float *src, int nb, int64_t V, float *dst) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < V * nb;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i % V;
        const int b = (int)(i / V);
        dst[i] = src[v * 4 + b];
    }
}

__global__ void k_zero4(float *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0f;
}

inline unsigned remapped_grid(int64_t n_slots) {  // windows, padded to a multiple of 8
    const int64_t nw = n_slots / kWindow;
    return (unsigned)((nw + 7) / 8 * 8);
}

hipError_t launch_otf_forward(const TabDesc &T, const double *tab, const RayDesc &rd,
                              const float *rho, int B, int64_t vf, float *y, hipStream_t st) {
    const int64_t V = vf * rd.n_obj_frames;  // voxels of all object frames
    const size_t sh = T.n_tab * sizeof(double);
    const dim3 grid(remapped_grid(rd.n_slots));
    float *vm = nullptr;
    if (B > 1) {
        hipError_t e = hipMallocAsync((void **)&vm, (size_t)V * 4 * sizeof(float), st);
        if (e != hipSuccess) return e;
    }
    for (int b0 = 0; b0 < B; b0 += 4) {
        const int nb = (B - b0 < 4) ? (B - b0) : 4;
        const float *r = rho + (int64_t)b0 * V;
        float *yy = y + (int64_t)b0 * rd.R;
        if (B == 1) {
            hipLaunchKernelGGL(k_otf_forward<1>, grid, dim3(256), sh, st, T, tab, rd, r, nb, V, yy);
        } else {
            hipLaunchKernelGGL(k_to_vmajor, dim3(strided_blocks(4 * V)), dim3(256), 0, st,
                               r, nb, V, vm);
            hipLaunchKernelGGL(k_otf_forward<4>, grid, dim3(256), sh, st, T, tab, rd, vm, nb, V,
                               yy);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return vm ? hipFreeAsync(vm, st) : hipSuccess;
}

// LDS of one adjoint workgroup: the grid tables, the hash table and the
// window's measurements.  Above 64 KiB (grids with large tables) a kernel
// must be allowed the size first.
template <int NB, bool FIX>
hipError_t otf_adjoint_lds(const TabDesc &T, size_t *sh) {
    *sh = (size_t)T.n_tab * sizeof(double) + OtfHash<NB, FIX>::kBytes +
          (size_t)kWindow * NB * sizeof(float);
    if (*sh <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void *)k_otf_adjoint<NB, FIX>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)*sh);
}

// x must be zero on entry for B == 1 (the caller clears it).
hipError_t launch_otf_adjoint(const TabDesc &T, const double *tab, const RayDesc &rd,
                              const float *y, int B, int64_t vf, float *x, hipStream_t st) {
    const int64_t V = vf * rd.n_obj_frames;  // voxels of all object frames
    size_t sh = 0;
    hipError_t e = B == 1 ? otf_adjoint_lds<1, false>(T, &sh) : otf_adjoint_lds<4, false>(T, &sh);
    if (e != hipSuccess) return e;
    const dim3 grid(remapped_grid(rd.n_slots));
    if (B == 1) {
        hipLaunchKernelGGL((k_otf_adjoint<1, false>), grid, dim3(256), sh, st, T, tab, rd, y, 1, V,
                           x, (unsigned long long *)nullptr, (const unsigned *)nullptr, 0.0);
        return hipGetLastError();
    }
    float *vm = nullptr;
    e = hipMallocAsync((void **)&vm, (size_t)V * 4 * sizeof(float), st);
    if (e != hipSuccess) return e;
    for (int b0 = 0; b0 < B; b0 += 4) {
        const int nb = (B - b0 < 4) ? (B - b0) : 4;
        const float *yy = y + (int64_t)b0 * rd.R;
        float *xx = x + (int64_t)b0 * V;
        hipLaunchKernelGGL(k_zero4, dim3(strided_blocks(4 * V)), dim3(256), 0, st, vm,
                           4 * V);
        hipLaunchKernelGGL((k_otf_adjoint<4, false>), grid, dim3(256), sh, st, T, tab, rd, yy, nb,
                           V, vm, (unsigned long long *)nullptr, (const unsigned *)nullptr, 0.0);
        hipLaunchKernelGGL(k_from_vmajor, dim3(strided_blocks(nb * V)), dim3(256), 0, st,
                           vm, nb, V, xx);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipFreeAsync(vm, st);
}

hipError_t launch_otf_adjoint_fixed(const TabDesc &T, const double *tab, const RayDesc &rd,
                                    const float *y, int B, int64_t vf, double r_out, float *x,
                                    hipStream_t st) {
    const int64_t V = vf * rd.n_obj_frames;
    const int NB = B == 1 ? 1 : 4;
    const double lsum = 2.0 * (double)rd.R * (2.0 * r_out);
    size_t sh = 0;
    hipError_t e = B == 1 ? otf_adjoint_lds<1, true>(T, &sh) : otf_adjoint_lds<4, true>(T, &sh);
    if (e != hipSuccess) return e;
    const dim3 grid(remapped_grid(rd.n_slots));
    // the sums, then four words of max |y|
    const int64_t words = V * NB + 2;
    unsigned long long *acc = nullptr;
    e = hipMallocAsync((void **)&acc, (size_t)words * 8, st);
    if (e != hipSuccess) return e;
    unsigned *bits = reinterpret_cast<unsigned *>(acc + V * NB);
    for (int b0 = 0; b0 < B; b0 += 4) {
        const int nb = (B - b0 < 4) ? (B - b0) : 4;
        const float *yy = y + (int64_t)b0 * rd.R;
        hipLaunchKernelGGL(k_zero_u64, dim3(strided_blocks(words)), dim3(256), 0, st,
                           acc, words);
        for (int b = 0; b < nb; b++) {
            e = launch_absmax(yy + (int64_t)b * rd.R, rd.R, bits + b, st);
            if (e != hipSuccess) break;
        }
        if (e != hipSuccess) break;
        if (B == 1)
            hipLaunchKernelGGL((k_otf_adjoint<1, true>), grid, dim3(256), sh, st, T, tab, rd, yy, 1,
                               V, (float *)nullptr, acc, bits, lsum);
        else
            hipLaunchKernelGGL((k_otf_adjoint<4, true>), grid, dim3(256), sh, st, T, tab, rd, yy, nb,
                               V, (float *)nullptr, acc, bits, lsum);
        hipLaunchKernelGGL(k_fix_to_float, dim3(strided_blocks(nb * V)), dim3(256), 0, st,
                           acc, NB, nb, V, bits, lsum, x + (int64_t)b0 * V);
        e = hipGetLastError();
        if (e != hipSuccess) break;
    }
    const hipError_t ef = hipFreeAsync(acc, st);
    return e != hipSuccess ? e : ef;
}

hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(k_zero_u64, dim3(strided_blocks(n)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_rays(const RayDesc &rd, double *starts, double *dirs, hipStream_t st) {
    hipLaunchKernelGGL(k_rays, dim3((unsigned)((rd.R + 255) / 256)), dim3(256), 0, st, rd, starts,
                       dirs);
    return hipGetLastError();
}

}  // namespace tsp
