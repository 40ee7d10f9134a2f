// Building the segment stores on gfx950: per-window ordering of ray slots,
// prefix sums, and the stable transposition of the ray-major segment lists
// into the voxel-major store used by the deterministic adjoint.
//
// Ray-major store ("sliced"): the 256 ray slots of a 16x16 detector window
// are ordered by decreasing segment count and cut into four 64-ray slices;
// slice s stores segment j of its lane l at sell_index(slice_ptr[s], l, j)
// (four consecutive segments per lane, 1 KiB per wavefront step), padded to
// the slice's longest list rounded up to 4.
//
// Voxel-major store: the canonical (ray-ordered) segments are sorted by voxel
// with a stable LSD radix sort (8-bit digits), so every voxel's list keeps
// increasing ray order and the adjoint sums it in a fixed order.  Voxels are
// keyed by store_key (all shells of one (e, a) cell together, the cells in
// 4 x 4 tiles): the rays through consecutive lists then form one compact fan
// per view, so the measurements they gather stay in L2 (in (r, e, a) order
// every shell needs nearly every ray).

#include "tsp_internal.h"

namespace tsp {
namespace {

// ------------------------------------------------------------ window sort

__global__ __launch_bounds__(256) void k_window_sort(RayDesc rd, const int32_t *cnt_nat,
                                                      int32_t *perm, int32_t *cnt_sorted,
                                                      int32_t *slice_len) {
    __shared__ uint64_t key[256];
    const int t = threadIdx.x;
    const int64_t slot = (int64_t)blockIdx.x * 256 + t;
    const int32_t ray = natural_ray(rd, slot);
    const int32_t c = cnt_nat[slot];
    // ascending key = (descending count, ascending ray, empty slots last)
    const uint32_t hi = 0x7fffffffu - (uint32_t)c;
    const uint32_t lo = (ray >= 0) ? (uint32_t)ray : 0xffffffffu;
    key[t] = ((uint64_t)hi << 32) | lo;
    __syncthreads();
    for (int k = 2; k <= 256; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int p = t ^ j;
            if (p > t) {
                const uint64_t a = key[t], b = key[p];
                const bool up = (t & k) == 0;
                if ((a > b) == up) {
                    key[t] = b;
                    key[p] = a;
                }
            }
            __syncthreads();
        }
    }
    const uint64_t mine = key[t];
    const int32_t cs = (int32_t)(0x7fffffffu - (uint32_t)(mine >> 32));
    const uint32_t r = (uint32_t)(mine & 0xffffffffu);
    perm[slot] = (r == 0xffffffffu) ? -1 : (int32_t)r;
    cnt_sorted[slot] = cs;
    if ((t & 63) == 0) slice_len[slot >> 6] = (cs + 3) & ~3;  // longest list, padded to 4
}

// ------------------------------------------------------------ scan (int32 -> int64)

constexpr int kScanItems = 8;
constexpr int kScanTile = 256 * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
    __shared__ int64_t ws[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int64_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) ws[w] = incl;
    __syncthreads();
    int64_t wpre = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        if (i < w) wpre += ws[i];
        tot += ws[i];
    }
    __syncthreads();
    *total = tot;
    return wpre + incl - v;
}

__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t *in, int64_t n, int64_t mul,
                                                      int64_t *blk) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++)
        if (base + i < n) s += (int64_t)in[base + i] * mul;
    int64_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) blk[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_scan_blocks(int64_t *blk, int64_t nb) {
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = (i < nb) ? blk[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, &tot);
        if (i < nb) blk[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) blk[nb] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t *in, int64_t n, int64_t mul,
                                                     const int64_t *blk, int64_t *out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        v[i] = (base + i < n) ? (int64_t)in[base + i] * mul : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t run = blk[blockIdx.x] + block_exclusive_scan(s, &tot);
#pragma unroll
    for (int i = 0; i < kScanItems; i++) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = blk[gridDim.x];
}

// ------------------------------------------------------------ canonical order

__global__ void k_scatter_nat(const RayDesc rd, const int32_t *seg_nat, int32_t *cnt_ray) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= rd.n_slots) return;
    const int32_t r = natural_ray(rd, slot);
    if (r >= 0) cnt_ray[r] = seg_nat[slot];
}

// Canonical CSR export: ray r's segments at row_ptr[r] ... in order, escape
// entries dropped.
__global__ __launch_bounds__(256) void k_expand(const RayDesc rd, const int32_t *perm,
                                                 const int32_t *cnt_sorted,
                                                 const int64_t *slice_ptr, const uint8_t *code,
                                                 const float *len, int64_t n_slots,
                                                 const int64_t *row_ptr, int na, int nena,
                                                 int32_t *out_vox, float *out_len) {
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;
    const int32_t r = perm[slot];
    if (r < 0) return;
    const int c = cnt_sorted[slot];
    const int64_t base = slice_ptr[slot >> 6];
    const int lane = (int)(slot & 63);
    int64_t dst = row_ptr[r];
    int32_t v = 0;
    for (int j = 0; j < c; j++) {
        const int64_t i = sell_index(base, lane, j);
        const int cd = code[i];
        const float l = decode_entry(cd, len[i], v, na, nena);
        if (cd == kCodeEsc) continue;
        if (out_vox) out_vox[dst] = v;
        if (out_len) out_len[dst] = l;
        dst++;
    }
}

// Voxel-major key of a segment of ray r in voxel v: object frame of the
// ray's view, then the voxel's store key.
__device__ __forceinline__ int32_t seg_key(const RayDesc &rd, int32_t r, int32_t v, int nr,
                                           int ne, int na) {
    return (int32_t)frame_base(rd.obj_frame, (int64_t)rd.H * rd.W, r, (int64_t)nr * ne * na) +
           store_key(v, nr, ne, na);
}

// Coarse histogram of the keys (bucket = key >> shift, nb <= kHistBuckets)
// over the ray-major store, to cut the transpose into passes of bounded size.
constexpr int kHistBuckets = 4096;
__global__ __launch_bounds__(256) void k_key_hist(const RayDesc rd, const int32_t *perm,
                                                   const int32_t *cnt_sorted,
                                                   const int64_t *slice_ptr, const uint8_t *code,
                                                   const float *len, int64_t n_slots, int nr, int ne, int na,
                                                   int shift, int nb,
                                                   unsigned long long *hist) {
    __shared__ unsigned h[kHistBuckets];
    for (int i = threadIdx.x; i < nb; i += 256) h[i] = 0;
    __syncthreads();
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot < n_slots) {
        const int32_t r = perm[slot];
        if (r >= 0) {
            const int c = cnt_sorted[slot];
            const int64_t base = slice_ptr[slot >> 6];
            const int lane = (int)(slot & 63);
            const uint32_t *cp = (const uint32_t *)(code + base) + lane;
            const float4 *lp = (const float4 *)(len + base) + lane;
            int32_t v = 0;
            for (int q = 0; q < ((c + 3) >> 2); q++) {
                const uint32_t cw = cp[(int64_t)q * kWave];
                const float4 lq = lp[(int64_t)q * kWave];
                const float la[4] = {lq.x, lq.y, lq.z, lq.w};
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    if (4 * q + e >= c) break;
                    const int cd = (cw >> (8 * e)) & 255;
                    decode_entry(cd, la[e], v, na, ne * na);
                    if (cd == kCodeEsc) continue;
                    atomicAdd(&h[seg_key(rd, r, v, nr, ne, na) >> shift], 1u);
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += 256)
        if (h[i]) atomicAdd(hist + i, (unsigned long long)h[i]);
}

// Per natural slot of a ray: number of its segments whose key lies in
// [lo, hi) (slots without a ray are left as they are: zero them first).
__global__ __launch_bounds__(256) void k_count_range(const RayDesc rd, const int32_t *perm,
                                                      const int32_t *cnt_sorted,
                                                      const int64_t *slice_ptr,
                                                      const uint8_t *code, const float *len,
                                                      int64_t n_slots,
                                                      int nr, int ne, int na, int32_t lo,
                                                      int32_t hi, int32_t *cnt_ray) {
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;
    const int32_t r = perm[slot];
    if (r < 0) return;
    const int c = cnt_sorted[slot];
    const int64_t base = slice_ptr[slot >> 6];
    const int lane = (int)(slot & 63);
    const int64_t nslot = natural_slot(rd, slot, r);
    const uint32_t *cp = (const uint32_t *)(code + base) + lane;
    const float4 *lp = (const float4 *)(len + base) + lane;
    int n = 0;
    int32_t v = 0;
    for (int q = 0; q < ((c + 3) >> 2); q++) {
        const uint32_t cw = cp[(int64_t)q * kWave];
        const float4 lq = lp[(int64_t)q * kWave];
        const float la[4] = {lq.x, lq.y, lq.z, lq.w};
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (4 * q + e >= c) break;
            const int cd = (cw >> (8 * e)) & 255;
            decode_entry(cd, la[e], v, na, ne * na);
            if (cd == kCodeEsc) continue;
            const int32_t k = seg_key(rd, r, v, nr, ne, na);
            n += (k >= lo && k < hi);
        }
    }
    cnt_ray[nslot] = n;
}

// Segments with keys in [lo, hi), compacted in natural slot order (the ray
// in natural slot s writes at crow[s] ...), as (key, natural slot | length
// bits << 32) for the sort: every key's entries then come out of the stable
// sort in increasing slot order.  A lane reads its ray's entries four at a
// time (one 4-byte code word, one 16-byte length load) and writes its items
// four at a time once its output is 16-byte aligned (16 bytes of keys, 32 of
// values per store group), single items at the head and tail of its run.
__global__ __launch_bounds__(256) void k_expand_range(const RayDesc rd, const int32_t *perm,
                                                       const int32_t *cnt_sorted,
                                                       const int64_t *slice_ptr,
                                                       const uint8_t *code, const float *len,
                                                       int64_t n_slots, const int64_t *crow,
                                                       int nr, int ne, int na, int32_t lo,
                                                       int32_t hi, int32_t *keys,
                                                       uint64_t *vals) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    typedef int v4i __attribute__((ext_vector_type(4)));
    typedef unsigned long long v2u __attribute__((ext_vector_type(2)));
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (slot >= n_slots) return;
    const int32_t r = perm[slot];
    if (r < 0) return;
    const int c = cnt_sorted[slot];
    const int64_t base = slice_ptr[slot >> 6];
    const int lane = (int)(slot & 63);
    const int64_t nslot = natural_slot(rd, slot, r);
    const uint64_t ns = (uint64_t)(uint32_t)nslot;
    const uint32_t *cp = (const uint32_t *)(code + base) + lane;
    const v4f *lp = (const v4f *)(len + base) + lane;
    int64_t dst = crow[nslot];
    int32_t v = 0;
    int nbuf = 0;
    int32_t k0 = 0, k1 = 0, k2 = 0, k3 = 0;
    uint64_t u0 = 0, u1 = 0, u2 = 0, u3 = 0;
    const int nq = (c + 3) >> 2;
    for (int q = 0; q < nq; q++) {
        const uint32_t cw = cp[(int64_t)q * kWave];
        const v4f lq = lp[(int64_t)q * kWave];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            if (4 * q + e >= c) break;
            const int cd = (cw >> (8 * e)) & 255;
            const float l = decode_entry(cd, lq[e], v, na, ne * na);
            if (cd == kCodeEsc) continue;
            const int32_t k = seg_key(rd, r, v, nr, ne, na);
            if (k < lo || k >= hi) continue;
            const uint64_t u = ns | ((uint64_t)__float_as_uint(l) << 32);
            if (nbuf == 0 && (dst & 3) != 0) {  // head of the run, before alignment
                keys[dst] = k;
                vals[dst] = u;
                dst++;
                continue;
            }
            k0 = nbuf == 0 ? k : k0;
            k1 = nbuf == 1 ? k : k1;
            k2 = nbuf == 2 ? k : k2;
            k3 = nbuf == 3 ? k : k3;
            u0 = nbuf == 0 ? u : u0;
            u1 = nbuf == 1 ? u : u1;
            u2 = nbuf == 2 ? u : u2;
            u3 = nbuf == 3 ? u : u3;
            if (++nbuf == 4) {
                *reinterpret_cast<v4i *>(keys + dst) = v4i{k0, k1, k2, k3};
                *reinterpret_cast<v2u *>(vals + dst) = v2u{u0, u1};
                *reinterpret_cast<v2u *>(vals + dst + 2) = v2u{u2, u3};
                dst += 4;
                nbuf = 0;
            }
        }
    }
    // the tail
    if (nbuf > 0) {
        keys[dst] = k0;
        vals[dst] = u0;
    }
    if (nbuf > 1) {
        keys[dst + 1] = k1;
        vals[dst + 1] = u1;
    }
    if (nbuf > 2) {
        keys[dst + 2] = k2;
        vals[dst + 2] = u2;
    }
}

// col_ptr[key0 + t] = base + (first index of keys >= key0 + t), t = 0..nk.
__global__ void k_col_ptr_range(const int32_t *keys, int64_t n, int64_t key0, int64_t nk,
                                int64_t base, int64_t *col_ptr) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > nk) return;
    const int64_t v = key0 + t;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    col_ptr[v] = base + lo;
}

// Packing of the sorted voxel-major lists (one wavefront per key).  Entry i
// of a list needs an escape before it when it is the list's first or when
// its slot increase over entry i - 1 exceeds kSlotMaxStep.
__device__ __forceinline__ bool needs_escape(int64_t i, int64_t lo, uint32_t slot,
                                             uint32_t prev) {
    return i == lo || slot - prev > (uint32_t)kSlotMaxStep;
}

// Rows of 64 entries that each key's packed list takes (escapes included).
__global__ __launch_bounds__(256) void k_pack_count(const int64_t *col_ptr, const uint64_t *ent,
                                                     int64_t nkeys, int32_t *rows) {
    const int lane = threadIdx.x & 63;
    // one key per wavefront; more only when the grid is capped
    for (int64_t key = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; key < nkeys;
         key += (int64_t)gridDim.x * 4) {
        const int64_t lo = col_ptr[key], hi = col_ptr[key + 1];
        int64_t n = 0;
        for (int64_t i = lo + lane; i < hi; i += kWave) {
            const uint32_t slot = (uint32_t)ent[i];
            const uint32_t prev = (i > lo) ? (uint32_t)ent[i - 1] : 0u;
            n += needs_escape(i, lo, slot, prev) ? 2 : 1;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, kWave);
        if (lane == 0) rows[key] = (int32_t)((n + kWave - 1) / kWave);
    }
}
__global__ __launch_bounds__(256) void k_pack_fill(const int64_t *col_ptr, const uint64_t *ent,
                                                    int64_t nkeys, const int64_t *base,
                                                    uint8_t *code, float *len) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // one key per wavefront; more only when the grid is capped
    for (int64_t key = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6; key < nkeys;
         key += (int64_t)gridDim.x * 4) {
        const int64_t lo = col_ptr[key], hi = col_ptr[key + 1];
        const int64_t p0 = base[key], p1 = base[key + 1];
        // entry q of the list (row q / 64, lane q % 64) is stored at p0 +
        // at(q): rows in groups of four interleaved (lane l's four entries
        // of a group contiguous), rows past the last whole group row-major
        const int64_t nq4 = ((p1 - p0) >> 8) << 8;
        auto at = [nq4](int64_t q) {
            return q < nq4 ? (q & ~(int64_t)255) + ((q & 63) << 2) + ((q >> 6) & 3) : q;
        };
        int64_t written = 0;
        for (int64_t c = lo; c < hi; c += kWave) {  // uniform over the wavefront
            const int64_t i = c + lane;
            const bool valid = i < hi;
            uint32_t slot = 0, prev = 0;
            float l = 0.0f;
            if (valid) {
                const uint64_t e = ent[i];
                slot = (uint32_t)e;
                l = __uint_as_float((uint32_t)(e >> 32));
                prev = (i > lo) ? (uint32_t)ent[i - 1] : 0u;
            }
            const bool esc = valid && needs_escape(i, lo, slot, prev);
            const uint64_t eb = __ballot(esc);
            const int64_t p = p0 + written + lane + __popcll(eb & below) + (esc ? 1 : 0);
            if (esc) {
                const int64_t pe = p0 + at(p - 1 - p0);
                code[pe] = (uint8_t)kSlotEsc;
                len[pe] = __uint_as_float(slot - prev);
            }
            if (valid) {
                const int64_t pv = p0 + at(p - p0);
                code[pv] = esc ? (uint8_t)0 : (uint8_t)(slot - prev);
                len[pv] = l;
            }
            written += __popcll(__ballot(valid)) + __popcll(eb);
        }
        for (int64_t q = written + lane; q < p1 - p0; q += kWave) {
            code[p0 + at(q)] = 0;
            len[p0 + at(q)] = 0.0f;
        }
    }
}

// x += a
__global__ void k_add(const float *a, float *x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) x[i] += a[i];
}

// dst[b][i] = src[b * stride + i], i < n, b < B
__global__ void k_copy_rows(const float *src, int64_t stride, float *dst, int64_t n, int B) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * B;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / n, k = i - b * n;
        dst[i] = src[b * stride + k];
    }
}

// ------------------------------------------------------------ radix sort

constexpr int kRsItems = 16;                // items per thread
constexpr int kRsTile = 256 * kRsItems;     // items per block
constexpr int kRsWaveItems = 64 * kRsItems;

__global__ __launch_bounds__(256) void k_rs_hist(const int32_t *keys, int64_t n, int shift,
                                                  int32_t *hist, int64_t nblk) {
    __shared__ unsigned cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int i = threadIdx.x; i < kRsTile; i += 256) {
        const int64_t idx = base + i;
        if (idx < n) atomicAdd(&cnt[(keys[idx] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = (int32_t)cnt[threadIdx.x];
}

// One digit pass of the stable LSD sort over a tile of kRsTile items, written
// straight to global memory: each wavefront ranks its items among equal
// digits (ballots over the 8 digit bits) and writes each item at its place.
// Used once the low digit is sorted: the higher digits of these keys are
// spatially coherent, so neighbouring items land close together anyway.
__global__ __launch_bounds__(256) void k_rs_scatter_direct(const int32_t *kin, const uint64_t *vin,
                                                     int32_t *kout, uint64_t *vout, int64_t n,
                                                     int shift, const int64_t *offs,
                                                     int64_t nblk) {
    __shared__ unsigned run[4][256];
    __shared__ unsigned wbase[4][256];
    __shared__ int64_t goff[256];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i < 1024; i += 256) (&run[0][0])[i] = 0;
    goff[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    __syncthreads();
    const int64_t wb = (int64_t)blockIdx.x * kRsTile + (int64_t)w * kRsWaveItems;
    for (int c = 0; c < kRsItems; c++) {
        const int64_t idx = wb + c * 64 + lane;
        if (idx < n) atomicAdd(&run[w][(kin[idx] >> shift) & 255], 1u);
    }
    __syncthreads();
    {
        unsigned acc = 0;
#pragma unroll
        for (int ww = 0; ww < 4; ww++) {
            const unsigned cc = run[ww][tid];
            wbase[ww][tid] = acc;
            acc += cc;
            run[ww][tid] = 0;
        }
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int c = 0; c < kRsItems; c++) {
        const int64_t idx = wb + c * 64 + lane;
        const bool valid = idx < n;
        const int32_t k = valid ? kin[idx] : 0;
        const uint64_t v = valid ? vin[idx] : 0ull;
        const int d = (k >> shift) & 255;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int bbit = 0; bbit < 8; bbit++) {
            const bool bitset = (d >> bbit) & 1;
            const uint64_t m = __ballot(bitset);
            match &= bitset ? m : ~m;
        }
        const unsigned rank = (unsigned)__popcll(match & below);
        const unsigned before = run[w][d];
        if (valid) {
            const int64_t pos = goff[d] + wbase[w][d] + before + rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        const bool leader = valid && ((match >> lane) == 1ull);
        __builtin_amdgcn_wave_barrier();
        if (leader) run[w][d] = before + (unsigned)__popcll(match);
        __builtin_amdgcn_wave_barrier();
    }
}

// The same pass with the tile reordered by digit in LDS first, so that each
// digit's run goes out contiguously at its place (goff, from the histogram
// scan) and global writes coalesce instead of scattering over 256 buckets:
// used for the lowest digit, which is spread at random over the input.  The
// tile (48 KB of items in LDS) is taken by eight wavefronts, so that two
// tiles fit a CU with 16 wavefronts between them.
constexpr int kTiledWaves = 8;
constexpr int kTiledThreads = 64 * kTiledWaves;
constexpr int kTiledItems = kRsTile / kTiledThreads;  // per thread
constexpr int kTiledWaveItems = 64 * kTiledItems;

__global__ __launch_bounds__(kTiledThreads) void k_rs_scatter_tiled(
    const int32_t *kin, const uint64_t *vin, int32_t *kout, uint64_t *vout, int64_t n, int shift,
    const int64_t *offs, int64_t nblk) {
    __shared__ unsigned run[kTiledWaves][256];
    __shared__ unsigned wbase[kTiledWaves][256];
    __shared__ unsigned loff[256];  // start of each digit within the tile
    __shared__ unsigned wsum[4];
    __shared__ int64_t goff[256];
    __shared__ int32_t lk[kRsTile];
    __shared__ uint64_t lv[kRsTile];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    for (int i = tid; i < kTiledWaves * 256; i += kTiledThreads) (&run[0][0])[i] = 0;
    if (tid < 256) goff[tid] = offs[(int64_t)tid * nblk + blockIdx.x];
    __syncthreads();
    const int64_t wb = (int64_t)blockIdx.x * kRsTile + (int64_t)w * kTiledWaveItems;
    for (int c = 0; c < kTiledItems; c++) {
        const int64_t idx = wb + c * 64 + lane;
        if (idx < n) atomicAdd(&run[w][(kin[idx] >> shift) & 255], 1u);
    }
    __syncthreads();
    // threads 0 .. 255 (wavefronts 0 .. 3) take one digit each
    unsigned tot = 0, incl = 0;  // items of digit tid in the tile, inclusive scan
    if (tid < 256) {
#pragma unroll
        for (int ww = 0; ww < kTiledWaves; ww++) {
            const unsigned cc = run[ww][tid];
            wbase[ww][tid] = tot;
            tot += cc;
            run[ww][tid] = 0;
        }
        incl = tot;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned t = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += t;
        }
        if (lane == 63) wsum[w] = incl;
    }
    __syncthreads();
    if (tid < 256) {
        unsigned wpre = 0;
        for (int ww = 0; ww < w; ww++) wpre += wsum[ww];
        loff[tid] = wpre + incl - tot;
    }
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int c = 0; c < kTiledItems; c++) {
        const int64_t idx = wb + c * 64 + lane;
        const bool valid = idx < n;
        const int32_t k = valid ? kin[idx] : 0;
        const uint64_t v = valid ? vin[idx] : 0ull;
        const int d = (k >> shift) & 255;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int bbit = 0; bbit < 8; bbit++) {
            const bool bitset = (d >> bbit) & 1;
            const uint64_t m = __ballot(bitset);
            match &= bitset ? m : ~m;
        }
        const unsigned rank = (unsigned)__popcll(match & below);
        const unsigned before = run[w][d];
        if (valid) {
            const unsigned p = loff[d] + wbase[w][d] + before + rank;
            lk[p] = k;
            lv[p] = v;
        }
        const bool leader = valid && ((match >> lane) == 1ull);
        __builtin_amdgcn_wave_barrier();
        if (leader) run[w][d] = before + (unsigned)__popcll(match);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const unsigned nvalid = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    for (unsigned i = tid; i < nvalid; i += kTiledThreads) {
        const int32_t k = lk[i];
        const int d = (k >> shift) & 255;
        const int64_t pos = goff[d] + (int64_t)(i - loff[d]);
        kout[pos] = k;
        vout[pos] = lv[i];
    }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_window_sort(const RayDesc &rd, const int32_t *cnt_nat, int32_t *perm,
                              int32_t *cnt_sorted, int32_t *slice_len, hipStream_t st) {
    hipLaunchKernelGGL(k_window_sort, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, rd,
                       cnt_nat, perm, cnt_sorted, slice_len);
    return hipGetLastError();
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan_i32(const int32_t *in, int64_t n, int64_t mul, int64_t *out,
                           int64_t *tmp, hipStream_t st) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, st, tmp, (int64_t)0);
        return hipMemcpyAsync(out, tmp, sizeof(int64_t), hipMemcpyDeviceToDevice, st);
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(256), 0, st, in, n, mul, tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, st, tmp, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(256), 0, st, in, n, mul,
                       (const int64_t *)tmp, out);
    return hipGetLastError();
}

hipError_t launch_scatter_nat(const RayDesc &rd, const int32_t *seg_nat, int32_t *cnt_ray,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_scatter_nat, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, rd,
                       seg_nat, cnt_ray);
    return hipGetLastError();
}

hipError_t launch_expand(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                         const int64_t *slice_ptr, const uint8_t *code, const float *len,
                         int64_t n_slots, const int64_t *row_ptr, int na, int nena,
                         int32_t *out_vox, float *out_len, hipStream_t st) {
    hipLaunchKernelGGL(k_expand, dim3(blocks_for(n_slots, 256)), dim3(256), 0, st, rd, perm,
                       cnt_sorted, slice_ptr, code, len, n_slots, row_ptr, na, nena, out_vox,
                       out_len);
    return hipGetLastError();
}

static int64_t rs_blocks(int64_t n) { return (n + kRsTile - 1) / kRsTile; }

size_t radix_ws_bytes(int64_t n) {
    const int64_t nb = rs_blocks(n);
    const int64_t h = 256 * nb;
    return sizeof(int32_t) * (size_t)h + sizeof(int64_t) * (size_t)(h + 1) +
           sizeof(int64_t) * (size_t)scan_tmp_elems(h) + 256;
}

hipError_t launch_radix_sort(int32_t *keys, uint64_t *vals, int32_t *keys2, uint64_t *vals2,
                             int64_t n, int key_bits, void *ws, int *in_second, hipStream_t st) {
    *in_second = 0;
    if (n <= 0) return hipSuccess;
    const int64_t nb = rs_blocks(n);
    const int64_t h = 256 * nb;
    char *p = (char *)ws;
    int32_t *hist = (int32_t *)p;
    p += sizeof(int32_t) * (size_t)h;
    p = (char *)(((uintptr_t)p + 15) & ~(uintptr_t)15);
    int64_t *offs = (int64_t *)p;
    p += sizeof(int64_t) * (size_t)(h + 1);
    int64_t *tmp = (int64_t *)p;
    int32_t *ka = keys, *kb = keys2;
    uint64_t *va = vals, *vb = vals2;
    int passes = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(256), 0, st, ka, n, shift, hist,
                           nb);
        hipError_t e = launch_scan_i32(hist, h, 1, offs, tmp, st);
        if (e != hipSuccess) return e;
        if (shift == 0)
            hipLaunchKernelGGL(k_rs_scatter_tiled, dim3((unsigned)nb), dim3(kTiledThreads), 0, st,
                               ka, va, kb,
                               vb, n, shift, offs, nb);
        else
            hipLaunchKernelGGL(k_rs_scatter_direct, dim3((unsigned)nb), dim3(256), 0, st, ka, va,
                               kb, vb, n, shift, offs, nb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        int32_t *tk = ka;
        ka = kb;
        kb = tk;
        uint64_t *tv = va;
        va = vb;
        vb = tv;
        passes++;
    }
    *in_second = passes & 1;
    return hipSuccess;
}

hipError_t launch_key_hist(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                           const int64_t *slice_ptr, const uint8_t *code, const float *len,
                           int nr, int ne, int na, int shift, int nb, unsigned long long *hist,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_key_hist, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, rd, perm,
                       cnt_sorted, slice_ptr, code, len, rd.n_slots, nr, ne, na, shift, nb, hist);
    return hipGetLastError();
}

hipError_t launch_count_range(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                              const int64_t *slice_ptr, const uint8_t *code, const float *len,
                              int nr, int ne, int na, int32_t lo, int32_t hi, int32_t *cnt_ray,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_count_range, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, rd,
                       perm, cnt_sorted, slice_ptr, code, len, rd.n_slots, nr, ne, na, lo, hi,
                       cnt_ray);
    return hipGetLastError();
}

hipError_t launch_expand_range(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                               const int64_t *slice_ptr, const uint8_t *code, const float *len,
                               const int64_t *crow, int nr, int ne, int na, int32_t lo,
                               int32_t hi, int32_t *keys, uint64_t *vals, hipStream_t st) {
    hipLaunchKernelGGL(k_expand_range, dim3(blocks_for(rd.n_slots, 256)), dim3(256), 0, st, rd,
                       perm, cnt_sorted, slice_ptr, code, len, rd.n_slots, crow, nr, ne, na, lo,
                       hi, keys, vals);
    return hipGetLastError();
}

hipError_t launch_col_ptr_range(const int32_t *sorted_keys, int64_t n, int64_t key0, int64_t nk,
                                int64_t base, int64_t *col_ptr, hipStream_t st) {
    hipLaunchKernelGGL(k_col_ptr_range, dim3(blocks_for(nk + 1, 256)), dim3(256), 0, st,
                       sorted_keys, n, key0, nk, base, col_ptr);
    return hipGetLastError();
}

hipError_t launch_pack_count(const int64_t *col_ptr, const uint64_t *ent, int64_t nkeys,
                             int32_t *m, hipStream_t st) {
    if (nkeys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_count, dim3(strided_blocks(nkeys * kWave)), dim3(256), 0, st,
                       col_ptr, ent, nkeys, m);
    return hipGetLastError();
}

hipError_t launch_pack_fill(const int64_t *col_ptr, const uint64_t *ent, int64_t nkeys,
                            const int64_t *base, uint8_t *code, float *len, hipStream_t st) {
    if (nkeys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack_fill, dim3(strided_blocks(nkeys * kWave)), dim3(256), 0, st,
                       col_ptr, ent, nkeys, base, code, len);
    return hipGetLastError();
}

hipError_t launch_add_f32(const float *a, float *x, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3(strided_blocks(n)), dim3(256), 0, st, a, x, n);
    return hipGetLastError();
}

hipError_t launch_copy_rows(const float *src, int64_t stride, float *dst, int64_t n, int B,
                            hipStream_t st) {
    if (n <= 0 || B <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_rows, dim3(strided_blocks(n * B)), dim3(256), 0, st, src, stride,
                       dst, n, B);
    return hipGetLastError();
}

}  // namespace tsp
