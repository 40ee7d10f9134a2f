// Internal declarations of the projector library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

namespace tsp {

constexpr int kWave = 64;     // CDNA wavefront
constexpr int kWindow = 256;  // ray slots per window: one 16x16 detector tile
constexpr int kTile = 16;
// One dispatch holds fewer than 2^32 work-items, and near the 2^31-voxel
// limit some launches have more items than that (four objects voxel-major,
// 64 lanes per voxel).  Those kernels take at most kMaxBlocks workgroups of
// 256 (2^31 work-items) and stride over the rest; smaller launches are
// unchanged.  max_blocks() is kMaxBlocks, or a smaller cap from the
// environment variable TSP_MAX_BLOCKS (read once per process), so that
// tests can make the striding run at small sizes.
constexpr int64_t kMaxBlocks = (int64_t)1 << 23;
int64_t max_blocks();
inline unsigned strided_blocks(int64_t items) {
    const int64_t b = (items + 255) / 256, cap = max_blocks();
    return (unsigned)(b < 1 ? 1 : (b > cap ? cap : b));
}

// Boundary tables (doubles) are staged in LDS: at most kMaxTabDoubles, so
// that they fit in 64 KiB per workgroup beside a 20 KiB hash table.  The
// on-the-fly adjoint's hash table takes at most kOtfHashBytes, and its
// launches ask for more than 64 KiB of LDS where a grid needs it (gfx950
// has 160 KiB per compute unit).
constexpr int kOtfHashBytes = 36864;
constexpr int kMaxTabDoubles = (65536 - 20480) / 8;

// Packed FP64 boundary tables, staged into LDS by every trace kernel.
//   rb[nr+1]    radii
//   ce[ne+1]    cos(e_b), decreasing
//   ca[np], sa[np]  cos/sin of the np distinct azimuth half-planes
//   ab[na+1]    a_b[k] - a_b[0]
struct TabDesc {
    double ab0;  // a_b[0]
    int nr, ne, na, np, cyclic;
    int off_rb, off_ce, off_ca, off_sa, off_ab, n_tab;
};

// Boundary tables of a validated grid (host): the descriptor and the packed
// values, in the layout above.  The grid is cyclic in azimuth when a_b spans
// 2 pi within 1e-12; then boundary na is boundary 0 and np = na half-planes
// remain, else np = na + 1.
inline void make_tables(const double *r_b, int nr, const double *e_b, int ne, const double *a_b,
                        int na, TabDesc *T, std::vector<double> *tab) {
    const double span = a_b[na] - a_b[0];
    const bool cyclic = std::fabs(span - 6.283185307179586476925286766559) <= 1e-12;
    const int np = cyclic ? na : na + 1;
    T->ab0 = a_b[0];
    T->nr = nr;
    T->ne = ne;
    T->na = na;
    T->np = np;
    T->cyclic = cyclic ? 1 : 0;
    T->off_rb = 0;
    T->off_ce = T->off_rb + nr + 1;
    T->off_ca = T->off_ce + ne + 1;
    T->off_sa = T->off_ca + np;
    T->off_ab = T->off_sa + np;
    T->n_tab = T->off_ab + na + 1;
    tab->assign((size_t)T->n_tab, 0.0);
    double *t = tab->data();
    for (int k = 0; k <= nr; k++) t[T->off_rb + k] = r_b[k];
    for (int k = 0; k <= ne; k++) t[T->off_ce + k] = std::cos(e_b[k]);
    for (int k = 0; k < np; k++) {
        t[T->off_ca + k] = std::cos(a_b[k]);
        t[T->off_sa + k] = std::sin(a_b[k]);
    }
    for (int k = 0; k <= na; k++) t[T->off_ab + k] = a_b[k] - a_b[0];
}

// Where rays come from: cone views (frames) or explicit arrays.
struct RayDesc {
    int n_views, H, W, tiles_h, tiles_w;
    int st;                // supertile side in tiles (divides tiles_h and tiles_w)
    // per view 16 doubles: pos(3) w(3) u(3) v(3) e_h e_w kind 0, where e_h / e_w
    // are tan(fov / 2) for a cone view (kind 0) and half the detector size for a
    // parallel view (kind 1)
    const double *frames;
    const double *starts;  // explicit: [R][3]
    const double *dirs;    // explicit: [R][3], unit
    int explicit_rays;
    int64_t R;
    int64_t n_slots;       // multiple of kWindow
    // dynamic objects: object frame of each cone view (device, [n_views]),
    // nullptr for a static object
    const int32_t *obj_frame;
    int n_obj_frames;      // 1 for a static object
};

// Offset, in voxels, of the object frame that ray r reads and writes: the
// frame of its view times the voxels of one frame (0 for a static object).
__host__ __device__ __forceinline__ int64_t frame_base(const int32_t *obj_frame, int64_t hw,
                                                       int32_t r, int64_t vf) {
    return obj_frame ? (int64_t)obj_frame[r / hw] * vf : 0;
}

// Slot -> ray id in the natural order: windows of 16x16 pixels of one view,
// enumerated supertile by supertile (st x st windows, row-major inside), so
// that consecutive windows cover a compact patch of the detector; each window
// is split into four 8x8 wavefront blocks; -1 for slots past the detector
// edge.  Explicit rays: slot i is ray i.
__device__ __forceinline__ int32_t natural_ray(const RayDesc &rd, int64_t slot) {
    if (rd.explicit_rays) return (slot < rd.R) ? (int32_t)slot : -1;
    const int64_t wdw = slot / kWindow;
    const int lane = (int)(slot % kWindow);
    const int per_view = rd.tiles_h * rd.tiles_w;
    const int view = (int)(wdw / per_view);
    const int t = (int)(wdw % per_view);
    const int st2 = rd.st * rd.st, sw = rd.tiles_w / rd.st;
    const int sidx = t / st2, inner = t % st2;
    const int ti = (sidx / sw) * rd.st + inner / rd.st;
    const int tj = (sidx % sw) * rd.st + inner % rd.st;
    const int w = lane >> 6, l = lane & 63;
    const int i = ti * kTile + (w >> 1) * 8 + (l >> 3);
    const int j = tj * kTile + (w & 1) * 8 + (l & 7);
    if (view >= rd.n_views || i >= rd.H || j >= rd.W) return -1;
    return (view * rd.H + i) * rd.W + j;
}

// Inverse of natural_ray inside one window: the natural slot of ray r, given
// any slot `in_window` of the window that holds it.  The voxel-major store
// keeps this slot rather than r, so that the adjoint gathers from a copy of y
// in slot order, where a 128-byte line holds a 4 x 8 pixel patch instead of
// 32 pixels of one detector row.
__host__ __device__ __forceinline__ int64_t natural_slot(const RayDesc &rd, int64_t in_window,
                                                         int32_t r) {
    if (rd.explicit_rays) return r;
    const int64_t hw = (int64_t)rd.H * rd.W;
    const int pix = (int)(r % hw);
    const int i = (pix / rd.W) & (kTile - 1), j = (pix % rd.W) & (kTile - 1);
    const int lane = (((i >> 3) << 1) | (j >> 3)) * 64 + (i & 7) * 8 + (j & 7);
    return (in_window & ~(int64_t)(kWindow - 1)) | lane;
}

// Ray-major store entries: a float32 length and a one-byte code.  Along a ray
// the next voxel almost always differs from the previous one by one step of
// one index (ir, ie or ia by +-1, ia wrapping round), so the code holds the
// step and the voxel index is rebuilt by a running sum:
//   0 stay (delta 0), 1 / 2 = +-1, 3 / 4 = +-na, 5 / 6 = +-ne*na,
//   7 / 8 = +-(na - 1) (an azimuth step across the cut of a cyclic grid),
//   kCodeEsc: the entry's length slot holds the next voxel index itself
//   (int32 bits) and the entry contributes nothing; the segment follows as a
//   "stay" entry.
// Every ray opens with an escape.  Padding entries are "stay" with length 0.
constexpr int kCodeEsc = 15;
__host__ __device__ __forceinline__ int32_t step_delta(int c, int na, int nena) {
    const int32_t mag = (c <= 2) ? 1 : (c <= 4) ? na : (c <= 6) ? nena : na - 1;
    return (c == 0 || c == kCodeEsc) ? 0 : ((c & 1) ? mag : -mag);
}
__host__ __device__ __forceinline__ int step_code(int32_t dv, int na, int nena) {
    if (dv == 0) return 0;
    if (dv == 1) return 1;
    if (dv == -1) return 2;
    if (dv == na) return 3;
    if (dv == -na) return 4;
    if (dv == nena) return 5;
    if (dv == -nena) return 6;
    if (dv == na - 1) return 7;
    if (dv == -(na - 1)) return 8;
    return kCodeEsc;
}
// One decoding step: updates the running voxel v, returns the segment length
// the entry carries (0 for an escape or padding).  The same deltas as
// step_delta, written as a chain of selects so that the decoder stays one
// branch-free run of instructions per entry (the compiler otherwise turns
// the range tests into branches around the gathers).
__device__ __forceinline__ float decode_entry(int c, float l, int32_t &v, int na, int nena) {
    const bool esc = c == kCodeEsc;
    int32_t mag = c >= 3 ? na : 1;
    mag = c >= 5 ? nena : mag;
    mag = c >= 7 ? na - 1 : mag;
    mag = (c == 0 || esc) ? 0 : mag;
    const int32_t delta = (c & 1) ? mag : -mag;
    const int32_t m = -(int32_t)esc;  // all ones for an escape
    v = (__float_as_int(l) & m) | ((v + delta) & ~m);
    return __int_as_float(__float_as_int(l) & ~m);
}

// Voxel-major store entries: a float32 length and a one-byte code.  Each
// (frame, voxel) list is sorted by natural slot; the code is the slot's
// increase over the previous entry's (0 ... 254) or kSlotEsc, an entry whose
// length slot carries the increase instead (uint32 bits) and that contributes
// nothing.  Every list opens with an escape (increase from slot 0) and is
// padded to whole rows of 64 entries with code 0, length 0; a wavefront takes
// a row at a time, lane l entry l, and rebuilds the slots by a prefix sum.
// In memory the rows sit in groups of four, interleaved (lane l's entries of
// a group adjacent: one 4-byte code word and one 16-byte length load per
// lane and group); rows past the last whole group stay row-major.
constexpr int kSlotEsc = 255;
constexpr int kSlotMaxStep = 254;

// Sum of x over the 64 lanes of a wavefront, returned to every lane: an
// inclusive scan by DPP (row shifts 1, 2, 4, 8 within rows of 16 lanes, then
// the broadcasts of lane 15 to rows 1 and 3 and of lane 31 to rows 2 and 3;
// lanes a step gives no source keep the old value 0), then lane 63.  Every
// lane must be active.
// Atomic scatters merge, per step, the lanes of a wavefront that hold the
// same voxel (one DPP sum and one global atomic per distinct voxel), for at
// most kMaxMerges distinct voxels; the lanes left over add directly.  A
// slice's lanes are rays sorted by segment count, not neighbours, and a step
// can touch dozens of voxels: past about 16 the merges cost more than the
// contention they save (stored atomic adjoint and attenuated backward at
// Medium: 16 best of 4, 8, 12, 16, 24, 32 and no limit).
constexpr int kMaxMerges = 16;

__device__ __forceinline__ float wave_sum_f32(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xf, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xa, 0xf, false));
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xc, 0xf, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Ray-major sliced store: slice s holds 64 rays (one per lane); segment j of
// lane l sits at slice_ptr[s] + 256 (j / 4) + 4 l + (j % 4), so each lane
// reads four consecutive segments with one 16-byte load and a wavefront reads
// 1 KiB contiguous.  Slices are padded to a multiple of 4 segments.
__host__ __device__ __forceinline__ int64_t sell_index(int64_t base, int lane, int j) {
    return base + (int64_t)(j >> 2) * 256 + lane * 4 + (j & 3);
}

// Voxel (ir, ie, ia) <-> its key in the voxel-major store: the (ie, ia)
// cells are taken in 4 x 4 tiles (row-major over tiles, row-major inside a
// tile, edge tiles partial), and all shells of one cell are consecutive.
// Consecutive keys are then voxels that every view sees in one compact patch
// of its detector, so the wavefronts working on them share cache lines of y.
constexpr int kKeyTile = 4;
__host__ __device__ __forceinline__ int32_t store_key(int32_t v, int nr, int ne, int na) {
    const int T = kKeyTile;
    const int ir = v / (ne * na), ie = (v / na) % ne, ia = v % na;
    const int te = ie / T, ta = ia / T;
    const int he = min(T, ne - te * T), ha = min(T, na - ta * T);
    const int cell = te * T * na + ta * he * T + (ie - te * T) * ha + (ia - ta * T);
    return cell * nr + ir;
}
__host__ __device__ __forceinline__ int32_t store_voxel(int64_t k, int nr, int ne,
                                                               int na) {
    const int T = kKeyTile;
    const int ir = (int)(k % nr);
    const int cell = (int)(k / nr);
    const int nte = (ne + T - 1) / T;
    const int te = min(cell / (T * na), nte - 1);
    const int rem = cell - te * T * na;
    const int he = min(T, ne - te * T);
    const int ta = rem / (he * T);
    const int rem2 = rem - ta * he * T;
    const int ha = min(T, na - ta * T);
    return (ir * ne + te * T + rem2 / ha) * na + ta * T + rem2 % ha;
}

// Events a launcher records on its stream around its main kernel (null:
// none); see tsp_set_timing_events.
struct KernelEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

// ---- launchers (tsp_trace.hip) ----
// win_seg (may be null, zeroed by the caller): canonical segments per window
// of kWindow natural slots
hipError_t launch_count(const TabDesc &T, const double *tab, const RayDesc &rd, int32_t *cnt_nat,
                        int32_t *seg_nat, unsigned long long *total, int *maxcnt,
                        int32_t *win_seg, hipStream_t st);
hipError_t launch_fill(const TabDesc &T, const double *tab, const RayDesc &rd,
                       const int32_t *perm, const int32_t *cnt_sorted, const int64_t *slice_ptr,
                       const int32_t *slice_len, uint8_t *code, float *len, int *err,
                       hipStream_t st);
// cnt_ray[natural_ray(s)] = seg_nat[s] for every natural slot s with a ray
hipError_t launch_scatter_nat(const RayDesc &rd, const int32_t *seg_nat, int32_t *cnt_ray,
                              hipStream_t st);
// vf: voxels of one object frame; rho / x hold rd.n_obj_frames frames per object.
hipError_t launch_otf_forward(const TabDesc &T, const double *tab, const RayDesc &rd,
                              const float *rho, int B, int64_t vf, float *y, hipStream_t st);
hipError_t launch_otf_adjoint(const TabDesc &T, const double *tab, const RayDesc &rd,
                              const float *y, int B, int64_t vf, float *x, hipStream_t st);
// The on-the-fly adjoint with reproducible sums in 64-bit fixed point
// (allocates its accumulators stream-ordered); r_out: outer radius.
hipError_t launch_otf_adjoint_fixed(const TabDesc &T, const double *tab, const RayDesc &rd,
                                    const float *y, int B, int64_t vf, double r_out, float *x,
                                    hipStream_t st);
hipError_t launch_rays(const RayDesc &rd, double *starts, double *dirs, hipStream_t st);

// p[0 .. n) = 0 (64-bit words), by a kernel
hipError_t launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st);
// *out = max |a[i]| over n floats, as float bits (atomicMax: *out zeroed first)
hipError_t launch_absmax(const float *a, int64_t n, unsigned *out, hipStream_t st);

// ---- launchers (tsp_sort.hip) ----
hipError_t launch_window_sort(const RayDesc &rd, const int32_t *cnt_nat, int32_t *perm,
                              int32_t *cnt_sorted, int32_t *slice_len, hipStream_t st);
// exclusive scan of n int32 values (times `mul`) into out[0..n] (int64, out[n] = total)
hipError_t launch_scan_i32(const int32_t *in, int64_t n, int64_t mul, int64_t *out,
                           int64_t *tmp, hipStream_t st);
int64_t scan_tmp_elems(int64_t n);
// Canonical CSR (ray-major, row_ptr order) export of the sliced store.
hipError_t launch_expand(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                         const int64_t *slice_ptr, const uint8_t *code, const float *len,
                         int64_t n_slots, const int64_t *row_ptr, int na, int nena,
                         int32_t *out_vox, float *out_len, hipStream_t st);
// stable LSD radix sort of (key, val) by key (key < 2^key_bits); result lands in
// (keys, vals) or (keys2, vals2): returns through *in_second whether it is the second.
hipError_t launch_radix_sort(int32_t *keys, uint64_t *vals, int32_t *keys2, uint64_t *vals2,
                             int64_t n, int key_bits, void *ws, int *in_second, hipStream_t st);
size_t radix_ws_bytes(int64_t n);
// Transpose in passes over key ranges [lo, hi) (bounded temporary memory):
// coarse key histogram (bucket = key >> shift, at most 4096 buckets),
// counts in a range per natural slot (cnt_ray: [n_slots], zeroed first),
// compacted expansion in natural slot order (crow: [n_slots + 1] offsets),
// and the range's column offsets with a base.
hipError_t launch_key_hist(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                           const int64_t *slice_ptr, const uint8_t *code, const float *len,
                           int nr, int ne, int na, int shift, int nb, unsigned long long *hist,
                           hipStream_t st);
hipError_t launch_count_range(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                              const int64_t *slice_ptr, const uint8_t *code, const float *len,
                              int nr, int ne, int na, int32_t lo, int32_t hi, int32_t *cnt_ray,
                              hipStream_t st);
hipError_t launch_expand_range(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                               const int64_t *slice_ptr, const uint8_t *code, const float *len,
                               const int64_t *crow, int nr, int ne, int na, int32_t lo,
                               int32_t hi, int32_t *keys, uint64_t *vals, hipStream_t st);
hipError_t launch_col_ptr_range(const int32_t *sorted_keys, int64_t n, int64_t key0, int64_t nk,
                                int64_t base, int64_t *col_ptr, hipStream_t st);
// x[i] += a[i], i < n
hipError_t launch_add_f32(const float *a, float *x, int64_t n, hipStream_t st);
// dst[b][i] = src[b * stride + i] for i < n, b < B (dst contiguous [B][n])
hipError_t launch_copy_rows(const float *src, int64_t stride, float *dst, int64_t n, int B,
                            hipStream_t st);
// Packing of the sorted voxel-major entries (col_ptr [nkeys + 1], ent =
// slot | length bits << 32): per key the rows of 64 entries its packed list
// takes, then the packed lists at base[key] (base = exclusive scan of 64 rows).
hipError_t launch_pack_count(const int64_t *col_ptr, const uint64_t *ent, int64_t nkeys,
                             int32_t *rows, hipStream_t st);
hipError_t launch_pack_fill(const int64_t *col_ptr, const uint64_t *ent, int64_t nkeys,
                            const int64_t *base, uint8_t *code, float *len, hipStream_t st);

// ---- launchers (tsp_apply.hip) ----
// vf: voxels of one object frame; rho / x hold rd.n_obj_frames frames per object.
hipError_t launch_forward_sell(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                               const int64_t *slice_ptr, const int32_t *slice_len,
                               const uint8_t *code, const float *len, const float *rho, int B,
                               int64_t vf, int na, int nena, float *y, hipStream_t st,
                               const KernelEvents *ke = nullptr);
// col_base is indexed by object frame, then the voxel's store key: the
// packed voxel-major store (codes and lengths, see kSlotEsc) of key k spans
// entries col_base[k] .. col_base[k+1]; x is written in (frame, r, e, a)
// order.  y is first copied into slot order (batch interleaved, groups of
// up to four objects in turn) in `ws`, adjoint_csc_ws_bytes(rd, B) bytes of
// device memory, or, when ws is null, in a stream-ordered temporary.
size_t adjoint_csc_ws_bytes(const RayDesc &rd, int B);
hipError_t launch_adjoint_csc(const RayDesc &rd, const int64_t *col_base, const uint8_t *code,
                              const float *len, int nr, int ne, int na, const float *y, int B,
                              float *x, void *ws, hipStream_t st,
                              const KernelEvents *ke = nullptr);
hipError_t launch_adjoint_atomic(const RayDesc &rd, const int32_t *perm,
                                 const int32_t *cnt_sorted, const int64_t *slice_ptr,
                                 const int32_t *slice_len, const uint8_t *code, const float *len,
                                 const float *y, int B, int64_t vf, int na, int nena, float *x,
                                 hipStream_t st);
hipError_t launch_zero_f32(float *p, int64_t n, hipStream_t st);

// ---- launchers (tsp_atten.hip): attenuated emission model, one object per
// launch of the line-of-sight kernels; arrays [B][V] / [B][R] ----
hipError_t launch_atten_s(const float *sigma, const float *rho, int64_t V, int B, float *s,
                          hipStream_t st);
hipError_t launch_atten_w(const float *tau1, const float *rho, int64_t n, float *w,
                          hipStream_t st);
hipError_t launch_atten_gtau(const float *w, const float *gw, int64_t n, float *out,
                             hipStream_t st);
hipError_t launch_atten_grad(const float *tau1, const float *sigma, const float *gw,
                             const float *gs, const float *gs_sun, int64_t V, int B, float *grad,
                             hipStream_t st);
hipError_t launch_fwd_atten(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                            const int64_t *slice_ptr, const int32_t *slice_len,
                            const uint8_t *code, const float *len, const float *s, const float *w,
                            int B, int64_t V, int na, int nena, float *y, hipStream_t st);
// gw, gs overwritten (zeroed by the caller when ws is null: float atomics);
// ws non-null: atten_fixed_ws_bytes(V) bytes for the fixed-point sums of the
// deterministic backward.  r_out: the grid's outer radius.
hipError_t launch_bwd_atten(const RayDesc &rd, const int32_t *perm, const int32_t *cnt_sorted,
                            const int64_t *slice_ptr, const int32_t *slice_len,
                            const uint8_t *code, const float *len, const float *s, const float *w,
                            const float *gy, int B, int64_t V, int na, int nena, double r_out,
                            float *gw, float *gs, void *ws, hipStream_t st);
size_t atten_fixed_ws_bytes(int64_t V);
hipError_t launch_copy_i64(const int64_t *src, int64_t *dst, int64_t n, hipStream_t st);

}  // namespace tsp
