// Step 4 of TomoSphero (Sec. 3.4, Eq. 5) and its adjoint from the stored
// segment lists, on gfx950.
//
// Forward: one lane per ray slot of a 64-ray slice of the ray-major store.
// Each lane reads four consecutive segments per 16-byte load (a wavefront
// reads 1 KiB contiguous of indices and of lengths), gathers rho (the object
// stays in L2), and accumulates len * rho in FP32 with FMA.  No reduction
// across lanes.
//
// Deterministic adjoint: one wavefront per voxel of the voxel-major store,
// fixed summation order, bitwise reproducible.
//
// Atomic adjoint: ray-major like the forward, scattering len * y into x with
// hardware float atomics, merged across the wavefront per voxel first.

#include "tsp_internal.h"

namespace tsp {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Streamed segment data is read once: non-temporal loads keep it from
// evicting the gathered object / measurements from L2.
__device__ __forceinline__ v4i ld_nt(const v4i *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ v4f ld_nt(const v4f *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ int32_t ld_nt(const int32_t *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ld_nt(const float *p) { return __builtin_nontemporal_load(p); }

// A batch lane group: NB = 1, 2 or 4 objects' values of one voxel (or one
// ray slot), loaded with one 4-, 8- or 16-byte access.
template <int NB> struct YVec;
template <> struct YVec<1> {
    using T = float;
    __device__ static float get(const T &v, int) { return v; }
    __device__ static void set(T &v, int, float f) { v = f; }
};
template <> struct YVec<2> {
    using T = float2;
    __device__ static float get(const T &v, int b) { return b ? v.y : v.x; }
    __device__ static void set(T &v, int b, float f) { (b ? v.y : v.x) = f; }
};
template <> struct YVec<4> {
    using T = float4;
    __device__ static float get(const T &v, int b) {
        return b == 0 ? v.x : b == 1 ? v.y : b == 2 ? v.z : v.w;
    }
    __device__ static void set(T &v, int b, float f) {
        (b == 0 ? v.x : b == 1 ? v.y : b == 2 ? v.z : v.w) = f;
    }
};

// Four entries of one lane: codes (one byte each, entry 0 lowest) and lengths.
template <int NB>
__device__ __forceinline__ void fwd_quad(uint32_t cw, const v4f l, int j, int c, int na,
                                         int nena, int32_t &v,
                                         const typename YVec<NB>::T *__restrict__ rho,
                                         float *acc) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const int cd = (cw >> (8 * i)) & 255;
        const float li = decode_entry(cd, l[i], v, na, nena);
        const bool ok = j + i < c && cd != kCodeEsc;  // escapes and padding add nothing
        const typename YVec<NB>::T r = rho[v];
#pragma unroll
        for (int b = 0; b < NB; b++) acc[b] = fmaf(li, ok ? YVec<NB>::get(r, b) : 0.0f, acc[b]);
    }
}

template <int NB>
__global__ __launch_bounds__(256) void k_fwd_sell(const int32_t *__restrict__ perm,
                                                   const int32_t *__restrict__ cnt_sorted,
                                                   const int64_t *__restrict__ slice_ptr,
                                                   const int32_t *__restrict__ slice_len,
                                                   const uint8_t *__restrict__ code,
                                                   const float *__restrict__ len, int64_t n_slots,
                                                   const typename YVec<NB>::T *__restrict__ rho,
                                                   int nb, int64_t R, float *__restrict__ y,
                                                   const int32_t *__restrict__ obj_frame,
                                                   int64_t hw, int64_t vf, int na, int nena) {
    // rho: voxel-major, NB objects per voxel (all object frames); vf: voxels of one frame
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;
    const int64_t s = slot >> 6;
    const int lane = (int)(slot & 63);
    const int32_t ray = perm[slot];
    rho += (ray >= 0) ? frame_base(obj_frame, hw, ray, vf) : 0;
    const int c = cnt_sorted[slot];
    const int nq = slice_len[s] >> 2;  // quads of segments in this slice
    const uint32_t *cp = (const uint32_t *)(code + slice_ptr[s]) + lane;
    const v4f *lp = (const v4f *)(len + slice_ptr[s]) + lane;
    int32_t v = 0;
    float acc[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) acc[b] = 0.0f;
    int q = 0;
    for (; q + 4 <= nq; q += 4) {
        uint32_t cw[4];
        v4f l[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            cw[u] = __builtin_nontemporal_load(cp + (int64_t)(q + u) * kWave);
            l[u] = ld_nt(lp + (int64_t)(q + u) * kWave);
        }
#pragma unroll
        for (int u = 0; u < 4; u++)
            fwd_quad<NB>(cw[u], l[u], 4 * (q + u), c, na, nena, v, rho, acc);
    }
    for (; q < nq; q++) {
        const uint32_t cw = __builtin_nontemporal_load(cp + (int64_t)q * kWave);
        const v4f l = ld_nt(lp + (int64_t)q * kWave);
        fwd_quad<NB>(cw, l, 4 * q, c, na, nena, v, rho, acc);
    }
    if (ray >= 0) {
#pragma unroll
        for (int b = 0; b < NB; b++)
            if (b < nb) y[b * R + ray] = acc[b];
    }
}

// dst[v] = (src[b][v] for b < nb), zero in unused lanes: a batch of objects
// packed voxel-major for the forward's gathers.
template <int NB>
__global__ void k_pack(const float *__restrict__ src, int nb, int64_t n,
                       typename YVec<NB>::T *__restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typename YVec<NB>::T v;
#pragma unroll
    for (int b = 0; b < NB; b++) YVec<NB>::set(v, b, b < nb ? src[b * n + i] : 0.0f);
    dst[i] = v;
}

// yt[s] = (y[b][natural_ray(s)] for b < nb), zero for padding slots and for
// the unused lanes of the last group.
template <int NB>
__global__ __launch_bounds__(256) void k_tile_y(const RayDesc rd, const float *__restrict__ y,
                                                 int nb, typename YVec<NB>::T *__restrict__ yt) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= rd.n_slots) return;
    const int32_t r = natural_ray(rd, s);
    typename YVec<NB>::T v;
#pragma unroll
    for (int b = 0; b < NB; b++) YVec<NB>::set(v, b, (r >= 0 && b < nb) ? y[b * rd.R + r] : 0.0f);
    yt[s] = v;
}

// Deterministic adjoint from the packed voxel-major store.
//
// Inclusive prefix sum over the 64 lanes of a wavefront: Hillis-Steele
// steps within rows of 16 lanes (DPP row shifts), then the broadcasts of
// lane 15 of each row to the next (rows 1 and 3) and of lane 31 to rows 2
// and 3.  Lanes that a step gives no source (the first k of a row for a
// shift by k, the rows outside the mask of a broadcast) keep the old value
// 0, the identity of the sum.  Every lane must be active.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// N rows of a packed voxel-major list (lane l: entry l of each row, its
// code and length loaded) into the lane sums; `run` is the slot before the
// first row.
template <int NB, int N>
__device__ __forceinline__ void adj_sum(const int *cd, const float *l, uint32_t smax,
                                        const typename YVec<NB>::T *__restrict__ yt,
                                        uint32_t &run, float *acc) {
    uint32_t sl[N];
#pragma unroll
    for (int u = 0; u < N; u++)
        sl[u] = wave_incl_sum(cd[u] == kSlotEsc ? __float_as_uint(l[u]) : (uint32_t)cd[u]);
#pragma unroll
    for (int u = 0; u < N; u++) {
        const uint32_t tot = __builtin_amdgcn_readlane(sl[u], 63);
        sl[u] += run;
        run += tot;
    }
#pragma unroll
    for (int u = 0; u < N; u++) {
        const bool ok = cd[u] != kSlotEsc && l[u] != 0.0f;  // escapes, padding: nothing
        const uint32_t si = sl[u] < smax ? sl[u] : smax;
        const typename YVec<NB>::T yv = yt[si];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const float t = fmaf(l[u], YVec<NB>::get(yv, b), acc[b]);
            acc[b] = ok ? t : acc[b];
        }
    }
}

// G groups of four interleaved rows: lane l's codes of the group's rows in
// one 4-byte word and its lengths in one 16-byte load (cg, lg: the group's
// first entry).
template <int NB, int G>
__device__ __forceinline__ void adj_groups(const uint8_t *__restrict__ cg,
                                           const float *__restrict__ lg, int lane, uint32_t smax,
                                           const typename YVec<NB>::T *__restrict__ yt,
                                           uint32_t &run, float *acc) {
    int cd[4 * G];
    float l[4 * G];
#pragma unroll
    for (int g = 0; g < G; g++) {
        const uint32_t w =
            __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(cg + g * 4 * kWave) + lane);
        const v4f v = ld_nt(reinterpret_cast<const v4f *>(lg + g * 4 * kWave) + lane);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            cd[4 * g + k] = (int)((w >> (8 * k)) & 255u);
            l[4 * g + k] = v[k];
        }
    }
    adj_sum<NB, 4 * G>(cd, l, smax, yt, run, acc);
}

// One row of the row-major tail (cp, lp: lane l's entry of the row).
template <int NB>
__device__ __forceinline__ void adj_row(const uint8_t *__restrict__ cp, const float *__restrict__ lp,
                                        uint32_t smax, const typename YVec<NB>::T *__restrict__ yt,
                                        uint32_t &run, float *acc) {
    const int cd = __builtin_nontemporal_load(cp);
    const float l = __builtin_nontemporal_load(lp);
    adj_sum<NB, 1>(&cd, &l, smax, yt, run, acc);
}

// Keys run over object frames, then voxels in store-key order; x is
// [nf][V] per object (nf = 1 for a static object).  One wavefront per key
// takes the key's packed list a row of 64 entries at a time (lane l entry
// l), eight rows in flight: each lane's slot is the running slot before the
// row plus the prefix sum of the row's increases (escapes carry theirs in
// the length slot).  The rows sit in groups of four, interleaved so that a
// lane's four codes are one 4-byte word and its four lengths 16 contiguous
// bytes; rows past the last whole group stay row-major.  A fixed butterfly adds the 64 lane sums, so the order
// never depends on timing: x is bitwise reproducible.
template <int NB>
__global__ __launch_bounds__(256) void k_adj_csc(const int64_t *__restrict__ col_base,
                                                  const uint8_t *__restrict__ code,
                                                  const float *__restrict__ len, int nr, int ne,
                                                  int na, int nf, int64_t n_slots,
                                                  const typename YVec<NB>::T *__restrict__ yt,
                                                  int nb, float *__restrict__ x) {
    constexpr int UNR = 8;
    const int64_t V = (int64_t)nr * ne * na;
    const int64_t FV = V * nf;
    // Workgroups reach the 8 XCDs round-robin.  Remap so that each XCD takes
    // chunks of 64 consecutive workgroups (256 consecutive keys) in turn: the
    // voxels of a chunk share y lines in that XCD's L2, while the chunks
    // still interleave finely enough to keep the XCDs' loads even.
    constexpr int64_t kChunk = 64;
    const int64_t nbk = gridDim.x, full = nbk / (8 * kChunk) * (8 * kChunk);
    const int64_t bx = blockIdx.x, q = bx / 8;
    const int64_t lb = (bx < full) ? ((q / kChunk) * 8 + bx % 8) * kChunk + q % kChunk : bx;
    // the key is uniform over the wavefront: keep it (and the list bounds,
    // the loop and the running slot) in scalar registers.  A wavefront takes
    // more than one key only when the grid is capped (more than 2^25 keys).
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    for (int64_t kb = lb; kb * 4 < FV; kb += nbk) {
        const int64_t key = kb * 4 + wv;
        if (key >= FV) break;
        const int64_t base = col_base[key];
        const int nrow = (int)((col_base[key + 1] - base) >> 6);
        const int64_t f = key / V;
        const int64_t v = f * V + store_voxel(key - f * V, nr, ne, na);
        const uint8_t *cb = code + base;
        const float *lb = len + base;
        const uint32_t smax = (uint32_t)(n_slots - 1);
        float acc[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) acc[b] = 0.0f;
        uint32_t run = 0;
        const int nrow4 = nrow & ~3;  // rows in interleaved groups of four
        int r = 0;
        for (; r + UNR <= nrow4; r += UNR)
            adj_groups<NB, UNR / 4>(cb + (int64_t)r * kWave, lb + (int64_t)r * kWave, lane, smax,
                                    yt, run, acc);
        for (; r < nrow4; r += 4)
            adj_groups<NB, 1>(cb + (int64_t)r * kWave, lb + (int64_t)r * kWave, lane, smax, yt,
                              run, acc);
        for (; r < nrow; r++)
            adj_row<NB>(cb + (int64_t)r * kWave + lane, lb + (int64_t)r * kWave + lane, smax, yt,
                        run, acc);
#pragma unroll
        for (int b = 0; b < NB; b++) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc[b] += __shfl_xor(acc[b], o, kWave);
        }
        if (lane == 0) {
#pragma unroll
            for (int b = 0; b < NB; b++)
                if (b < nb) x[b * FV + v] = acc[b];
        }
    }
}

// Atomic adjoint from the ray-major store.  The 64 rays of a slice (one 16x16
// detector window) cross similar voxels; each step the wavefront takes the
// j-th segment of every lane, adds up the contributions that land in the same
// voxel, and one lane per distinct voxel issues the atomic add (for up to
// kMaxMerges distinct voxels; the rest add directly).
template <int NB>
__global__ __launch_bounds__(256) void k_adj_atomic(const int32_t *__restrict__ perm,
                                                     const int32_t *__restrict__ cnt_sorted,
                                                     const int64_t *__restrict__ slice_ptr,
                                                     const int32_t *__restrict__ slice_len,
                                                     const uint8_t *__restrict__ code,
                                                     const float *__restrict__ len,
                                                     int64_t n_slots, const float *__restrict__ y,
                                                     int nb, int64_t V, int64_t R, float *x,
                                                     const int32_t *__restrict__ obj_frame,
                                                     int64_t hw, int64_t vf, int na, int nena) {
    // V: batch stride of x (voxels of all object frames); vf: one frame
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;  // n_slots is a multiple of 256: whole wavefronts
    const int lane = (int)(slot & 63);
    const int32_t ray = perm[slot];
    const int32_t fb = (ray >= 0) ? (int32_t)frame_base(obj_frame, hw, ray, vf) : 0;
    const int c = (ray >= 0) ? cnt_sorted[slot] : 0;
    const int m = slice_len[slot >> 6];
    const int64_t base = slice_ptr[slot >> 6];
    float yv[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) yv[b] = (ray >= 0 && b < nb) ? y[b * R + ray] : 0.0f;
    int32_t vraw = 0;
    const uint32_t *cp = (const uint32_t *)(code + base) + lane;
    const v4f *lp = (const v4f *)(len + base) + lane;
    for (int q = 0; q < (m >> 2); q++) {  // m is uniform over the wavefront, a multiple of 4
        const uint32_t cw = __builtin_nontemporal_load(cp + (int64_t)q * kWave);
        const v4f lq = ld_nt(lp + (int64_t)q * kWave);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            int v = -1;
            float l = 0.0f;
            if (4 * q + e < c) {
                const int cd = (cw >> (8 * e)) & 255;
                l = decode_entry(cd, lq[e], vraw, na, nena);
                v = (cd == kCodeEsc) ? -1 : fb + vraw;
            }
            float cb[NB];
#pragma unroll
            for (int b = 0; b < NB; b++) cb[b] = (v >= 0) ? l * yv[b] : 0.0f;
            uint64_t pend = __ballot(v >= 0);
            // uniform over the wavefront: every lane is active
            for (int it = 0; pend && it < kMaxMerges; it++) {
                const int leader = __ffsll((unsigned long long)pend) - 1;
                const int v0 = __builtin_amdgcn_readlane(v, leader);
                const bool mine = (v == v0);
#pragma unroll
                for (int b = 0; b < NB; b++) {
                    const float sb = wave_sum_f32(mine ? cb[b] : 0.0f);
                    if (lane == leader && b < nb) atomicAdd(x + b * V + v0, sb);
                }
                pend &= ~__ballot(mine);
            }
            if ((pend >> lane) & 1ull) {  // past the merge limit
#pragma unroll
                for (int b = 0; b < NB; b++)
                    if (b < nb) atomicAdd(x + b * V + v, cb[b]);
            }
        }
    }
}

__global__ void k_zero(float *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) p[i] = 0.0f;
}

__global__ void k_copy_i64(const int64_t *s, int64_t *d, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) d[i] = s[i];
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// Records ev on st when it is set (the timing events around a main kernel).
static hipError_t record_if(hipEvent_t ev, hipStream_t st) {
    return ev ? hipEventRecord(ev, st) : hipSuccess;
}

template <int NB>
static hipError_t fwd_chunk(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                            const int64_t *slice_ptr, const int32_t *slice_len,
                            const uint8_t *code, const float *len, const float *rho, int nb,
                            int64_t vf, int64_t FV, int na, int nena, float *y, void *packed,
                            hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
    using T = typename YVec<NB>::T;
    const T *r = (const T *)rho;
    if (NB > 1) {
        hipLaunchKernelGGL(k_pack<NB>, dim3(blocks_for(FV, 256)), dim3(256), 0, st, rho, nb, FV,
                           (T *)packed);
        r = (const T *)packed;
    }
    hipError_t e = record_if(ev_start, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fwd_sell<NB>, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, perm,
                       cnt_sorted, slice_ptr, slice_len, code, len, rd.n_slots, r, nb, rd.R, y,
                       rd.obj_frame, (int64_t)rd.H * rd.W, vf, na, nena);
    e = hipGetLastError();
    return e != hipSuccess ? e : record_if(ev_stop, st);
}

hipError_t launch_forward_sell(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                               const int64_t *slice_ptr, const int32_t *slice_len,
                               const uint8_t *code, const float *len, const float *rho, int B,
                               int64_t vf, int na, int nena, float *y, hipStream_t st,
                               const KernelEvents *ke) {
    // batches: objects packed voxel-major (4, 8 or 16 bytes per voxel) so that
    // one gather per segment serves every object of a group of up to four
    const int64_t FV = vf * rd.n_obj_frames;
    const int width = B >= 3 ? 4 : B;
    void *packed = nullptr;
    hipError_t e = hipSuccess;
    if (B > 1) {
        e = hipMallocAsync(&packed, (size_t)FV * width * sizeof(float), st);
        if (e != hipSuccess) return e;
    }
    for (int b0 = 0; b0 < B && e == hipSuccess; b0 += 4) {
        const int nb = (B - b0 < 4) ? (B - b0) : 4;
        const float *r = rho + (int64_t)b0 * FV;
        float *yy = y + (int64_t)b0 * rd.R;
        // the timing events go round the first group's kernel to the last's
        const hipEvent_t es = (ke && b0 == 0) ? ke->start : nullptr;
        const hipEvent_t ee = (ke && b0 + 4 >= B) ? ke->stop : nullptr;
        if (nb == 1)
            e = fwd_chunk<1>(rd, perm, cnt_sorted, slice_ptr, slice_len, code, len, r, nb, vf,
                             FV, na, nena, yy, packed, st, es, ee);
        else if (nb == 2)
            e = fwd_chunk<2>(rd, perm, cnt_sorted, slice_ptr, slice_len, code, len, r, nb, vf,
                             FV, na, nena, yy, packed, st, es, ee);
        else
            e = fwd_chunk<4>(rd, perm, cnt_sorted, slice_ptr, slice_len, code, len, r, nb, vf,
                             FV, na, nena, yy, packed, st, es, ee);
    }
    if (packed) {
        const hipError_t f = hipFreeAsync(packed, st);
        if (e == hipSuccess) e = f;
    }
    return e;
}

template <int NB>
static hipError_t adj_csc_chunk(const RayDesc &rd, const int64_t *col_base, const uint8_t *code,
                                const float *len, int nr, int ne, int na, const float *y,
                                int nb, float *x, void *yt, hipStream_t st, hipEvent_t ev_start,
                                hipEvent_t ev_stop) {
    using T = typename YVec<NB>::T;
    const int64_t FV = (int64_t)nr * ne * na * rd.n_obj_frames;
    hipLaunchKernelGGL(k_tile_y<NB>, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, rd, y,
                       nb, (T *)yt);
    hipError_t e = record_if(ev_start, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_csc<NB>, dim3(strided_blocks(FV * kWave)), dim3(256), 0, st,
                       col_base, code, len, nr, ne, na, rd.n_obj_frames, rd.n_slots,
                       (const T *)yt, nb, x);
    e = hipGetLastError();
    return e != hipSuccess ? e : record_if(ev_stop, st);
}

size_t adjoint_csc_ws_bytes(const RayDesc &rd, int B) {
    const int width = B >= 3 ? 4 : B;
    return (size_t)rd.n_slots * width * sizeof(float);
}

hipError_t launch_adjoint_csc(const RayDesc &rd, const int64_t *col_base, const uint8_t *code,
                              const float *len, int nr, int ne, int na, const float *y, int B,
                              float *x, void *ws, hipStream_t st, const KernelEvents *ke) {
    const int64_t FV = (int64_t)nr * ne * na * rd.n_obj_frames;
    void *yt = ws;
    hipError_t e = hipSuccess;
    if (!ws) {
        e = hipMallocAsync(&yt, adjoint_csc_ws_bytes(rd, B), st);
        if (e != hipSuccess) return e;
    }
    for (int b0 = 0; b0 < B && e == hipSuccess; b0 += 4) {
        const int nb = (B - b0 < 4) ? (B - b0) : 4;
        const float *yy = y + (int64_t)b0 * rd.R;
        float *xx = x + (int64_t)b0 * FV;
        const hipEvent_t es = (ke && b0 == 0) ? ke->start : nullptr;
        const hipEvent_t ee = (ke && b0 + 4 >= B) ? ke->stop : nullptr;
        if (nb == 1)
            e = adj_csc_chunk<1>(rd, col_base, code, len, nr, ne, na, yy, nb, xx, yt, st, es, ee);
        else if (nb == 2)
            e = adj_csc_chunk<2>(rd, col_base, code, len, nr, ne, na, yy, nb, xx, yt, st, es, ee);
        else
            e = adj_csc_chunk<4>(rd, col_base, code, len, nr, ne, na, yy, nb, xx, yt, st, es, ee);
    }
    if (ws) return e;
    const hipError_t f = hipFreeAsync(yt, st);
    return e != hipSuccess ? e : f;
}

hipError_t launch_adjoint_atomic(const RayDesc &rd, const int32_t *perm,
                                 const int32_t *cnt_sorted, const int64_t *slice_ptr,
                                 const int32_t *slice_len, const uint8_t *code, const float *len,
                                 const float *y, int B, int64_t vf, int na, int nena, float *x,
                                 hipStream_t st) {
    const int64_t FV = vf * rd.n_obj_frames, R = rd.R, hw = (int64_t)rd.H * rd.W;
    const int64_t n_slots = rd.n_slots;
    for (int b0 = 0; b0 < B; b0 += 4) {
        const int nb = (B - b0 < 4) ? (B - b0) : 4;
        const float *yy = y + (int64_t)b0 * R;
        float *xx = x + (int64_t)b0 * FV;
        const dim3 g(blocks_for(n_slots, 256));
        if (nb == 1)
            hipLaunchKernelGGL(k_adj_atomic<1>, g, dim3(256), 0, st, perm, cnt_sorted, slice_ptr,
                               slice_len, code, len, n_slots, yy, nb, FV, R, xx, rd.obj_frame, hw,
                               vf, na, nena);
        else if (nb == 2)
            hipLaunchKernelGGL(k_adj_atomic<2>, g, dim3(256), 0, st, perm, cnt_sorted, slice_ptr,
                               slice_len, code, len, n_slots, yy, nb, FV, R, xx, rd.obj_frame, hw,
                               vf, na, nena);
        else
            hipLaunchKernelGGL(k_adj_atomic<4>, g, dim3(256), 0, st, perm, cnt_sorted, slice_ptr,
                               slice_len, code, len, n_slots, yy, nb, FV, R, xx, rd.obj_frame, hw,
                               vf, na, nena);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(strided_blocks(n)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_copy_i64(const int64_t *src, int64_t *dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_i64, dim3(strided_blocks(n)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

}  // namespace tsp
