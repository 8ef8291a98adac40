// Kernel argument blocks and launcher entry points shared by the host API
// (prt_api.cpp) and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.hpp"

namespace prt {

// Device view of a path store in wavefront-batch layout: sorted slot i
// belongs to batch i/64, lane i%64; vertex k of that slot is the float4
// record vtx[batch_off[i/64] + 64*k + i%64] = (x, y, z, voxel bits), grid units.
struct StoreView {
    const float4* vtx;
    const int64_t* batch_off;
    const uint8_t* B;       // scatters per sorted slot
    const uint8_t* nv;      // stored vertices per sorted slot (0 for padding)
    int64_t n_slots;        // 64 * n_batches
    int64_t first_slot;     // first slot with B > 0 (sorted order)
    const float* beta_ref;  // reference cloud field
};

// Where the sampler puts a path's vertex records: row id of tmp (one-pass
// resample; tmp has max_order+2 records per path), straight into the packed
// store (vtx non-null: the second pass of a two-pass resample, slot = inv[id],
// vertex k at vtx[batch_off[slot/64] + 64 k + slot%64]), or nowhere (both
// null: the first pass of a two-pass resample, which only records sizes and
// sort keys).  The second pass draws the same paths again from the same
// Philox streams with the same code; it checks each path's size against the
// first pass's and sets *mismatch otherwise.
// Overflow segment of a short-row draw: 128 bytes, one cache line.
constexpr int kSegRecords = 8;

struct SampleArgs {
    DevScene s;
    const float* beta_c;   // cloud field the paths are drawn from
    const void* grid_tot;  // Real[N_u]: beta_c + beta_air
    const void* grid_tile; // the same in the z-tiled layout (walked when the grid is read from global memory)
    uint64_t seed;
    int64_t n;
    float4* tmp;           // [n][tmp_rows] records, or null
    // Short temporary rows (tmp_rows < max_order+2): a path's records from
    // tmp_rows on go to a chain of segments of the overflow pool
    // (kSegRecords float4 each: kSegRecords-1 records, then the next
    // segment's index as an int in .x); the first segment's index is
    // ovf_slot[id].  Wavefronts claim segments in chunks of ovf_chunk from
    // *ovf_next (a segment count); a path that finds the ovf_cap segments
    // used up sets *ovf_full and stores no more.
    int tmp_rows;
    int ovf_chunk;
    float4* ovf;
    int64_t ovf_cap;
    unsigned long long* ovf_next;
    int32_t* ovf_slot;
    int* ovf_full;
    float4* vtx;           // packed store records, or null
    const int64_t* batch_off;
    const int32_t* inv;    // path id -> sorted slot
    int* mismatch;
    uint8_t* tB;
    uint8_t* tnv;
    uint16_t* tC;          // spatial sort key per path (cell_key)
    unsigned int* next;    // path-id counter of the persistent sampler (zero at launch)
};

// Task counters of the persistent kernels.  One atomic counter serialises
// every wavefront's task requests on one address; a launch therefore spreads
// its tasks over kTaskCounters counters on separate 128-byte lines, and a
// context holds kWorkWords words of them (render/grad counters at word 0 and
// 1 of each line, the sampler's id counter at word 2 of the first).
constexpr int kTaskCounters = 8;
constexpr int kTaskStride = 32;
constexpr int kWorkWords = kTaskCounters * kTaskStride;

struct TraceArgs {
    DevScene s;
    StoreView st;
    const float* bc_t;        // current cloud field
    const void* grid_tot;     // Real[N_u]: beta_t + beta_air
    const void* grid_dlt;     // Real[N_u]: beta_t - beta_ref
    const void* grid_tile;    // grid_tot in the z-tiled layout (tile_index), for the render's walks
    double* img;              // render: raw tallies [n][H][W]
    const double* rho;        // grad: residual / (N Omega_p) [n][H][W]
    double* grad;             // grad: [N_u]
    double* partial;          // reweight: per-block (sum r, sum r^2)
    int32_t brender;
    unsigned long long* counters;  // [0] voxel segs, [1] local estimates, [3] overhead segs
    // Transmittance tape: render records, for every (scatter b, camera d),
    // (c_{b,d}, pixel index as int bits), or (0, -1) when x_b projects outside
    // camera d, at tape[(batch_off[batch] - tape_base) * n_cams + (b*n_cams + d)*64 + lane];
    // grad reuses it when *tape_flag is 1 (same beta_t, cameras and scene).
    float2* tape;
    int64_t tape_base;        // records of the leading batches without scatters
    // Render prefix: pbase[batch_off[batch] - tape_base + 64*b + lane] =
    // base_b / base_{b-1} (base_0 = 1), base_b = P_b / (beta_ref(x_b) +
    // beta_air) being the recycled weight of the sub-path x_0..x_b without its
    // last direction factor and connection.
    double* pbase;
    const int* tape_flag;
    // Gradient weights (tape case): wtape has the tape's layout and holds
    // w_{b,d} = c_{b,d} rho_{d,p} (0 outside the image); vaux[batch_off[batch] -
    // tape_base + 64*b + lane] = (R_b, connection vertex term at x_b,
    // w_c f_HG / f_s,t of the scatter at x_b, 0).
    float* wtape;
    float4* vaux;
    // Dynamic schedule: wavefront w takes tasks from the counter
    // work[(w % kTaskCounters) * kTaskStride] (reset to 0 before the launch),
    // which hands out tasks c, c + kTaskCounters, c + 2 kTaskCounters, ... for
    // c = w % kTaskCounters; task t covers batch n_batches-1-t/groups
    // (heaviest first, the batches being sorted by size) and camera group
    // t%groups.
    unsigned int* work;
    int groups;
    // render prefix: also copies beta_t here (the tape's field) when set, and
    // zeroes the render's task counters
    float* copy_beta;
    // Binned gradient (tape case): trange[2*t], trange[2*t+1] = first and last
    // slab that a walk of gradient task t reaches (t numbered as in the walk
    // kernels: batch n_batches-1-t/(groups+1), kind t%(groups+1)); set by the
    // weights kernel when non-null.
    int* trange;
    int bin_axis, bin_layers;  // slab axis and layers per slab of those ranges
    // and, per connection, its own slab range lo | hi << 8 in the tape's
    // layout (0xffff when the connection has no weight: lo = 255 exceeds
    // every slab)
    uint16_t* rtape;
    // and, per row of 64 records (tape row r = record / 64) and camera group
    // g, the union of that row's connection ranges at brange[r * groups + g]
    // (0xffff when the row has no weighted connection in the group)
    uint32_t* brange;
};

// Slabs of the binned gradient: layers of the grid along `axis`, `layers`
// per slab (the last one may be thinner), each slab tallied in LDS with its
// voxels numbered (i_b + n_b (i_c + n_c (i_axis - first layer))), b < c the
// other two axes.
struct GradBins {
    int axis;
    int layers;
    int n_slabs;
    int64_t n_tasks;     // (batches from the first scattering one) * (groups + 1)
    int64_t n_blocks;    // blocks of kBinTasks tasks
    uint32_t* cnt;       // [n_slabs * n_blocks + 1], scanned in place
    uint32_t* list;      // task ids, slab after slab
    int64_t list_cap;
    uint32_t* chunks;    // [n_slabs + 2]: first chunk of each slab, chunk count, chunk size
    double* partial;     // per chunk: the slab's sums
};
constexpr int kBinTasks = 1024;
// slabs the binning kernels count per block; a connection's slab range
// packs two slab indices into 8 bits each
constexpr int kMaxBinSlabs = 255;
constexpr int kBinChunkWord = 3;  // chunk counter of the binned walk: word 3 of the task-counter set

// Per-vertex task levels of the render prefix and the gradient weights: one
// task per (batch, scatter index b) with a path of at least b scatters.  The
// store is sorted by B, so the batches of level b are [first_batch[b],
// n_batches); levels run from b = bmax down to 1, level b's tasks start at
// start[b], and total counts them all.
struct VertexLevels {
    int bmax;
    uint32_t total;
    int32_t first_batch[kMaxOrder + 1];
    uint32_t start[kMaxOrder + 1];
};

// ---- sampling, sorting, packing (sample.hip)
// grid_tot = beta_t + beta_air and grid_dlt = beta_t - beta_ref in the
// traversal precision (each when given); also copy = beta_t and *zero = 0
// when given, and grid_tot in the z-tiled layout of an nx x ny grid
// (tile_index) into tile when given.
hipError_t launch_prep_grids(hipStream_t st, int fp64, const float* bc_t, const float* bc_r, double beta_air,
                             int64_t nu, void* grid_tot, void* grid_dlt, float* copy = nullptr,
                             unsigned int* zero = nullptr, void* tile = nullptr, int nx = 0, int ny = 0);
hipError_t launch_sample(hipStream_t st, int fp64, const SampleArgs& a, int n_cu);
// Stable sort of the paths by (size B, spatial key): perm[sorted position] =
// path id, B[position] = size, nv[position] = tnv[path id] for positions < n
// and 0 up to n_slots, and (when inv is given) inv[path id] = sorted position.
// hist: sort_scratch_words(n, nbins) words; tmp_perm and carry: n entries.
hipError_t launch_sort_paths(hipStream_t st, const uint8_t* size_key, const uint8_t* tnv, const uint16_t* cell,
                             int64_t n, int64_t n_slots, int nbins, uint32_t* hist, int32_t* tmp_perm,
                             uint16_t* carry, int32_t* perm,
                             uint8_t* B, uint8_t* nv, int32_t* inv);
int64_t sort_scratch_words(int64_t n, int nbins);
// scratch: the sort's scratch (sort_scratch_words(64 * nb, ...) words) may be reused.
hipError_t launch_batch_offsets(hipStream_t st, const uint8_t* nv, int64_t nb, int64_t* batch_off, void* scratch);
// Record k of the path in slot i: tmp[(tmp_off ? tmp_off[id] : id * tmp_stride) + k],
// or, with an overflow pool and k >= tmp_stride, record (k - tmp_stride) of
// the chain of segments that starts at ovf_slot[id] (SampleArgs).
hipError_t launch_pack(hipStream_t st, const int32_t* perm, const float4* tmp, const int64_t* tmp_off,
                       int64_t tmp_stride, const uint8_t* nv, const int64_t* batch_off, int64_t n,
                       int64_t n_slots, float4* vtx, const float4* ovf = nullptr, const int32_t* ovf_slot = nullptr);
// meta[0] = batch_off[nb] (records), meta[1] = first slot with B > 0 (n if
// none), meta[2] = batch_off of that slot's batch (records of B = 0 batches),
// meta[kMetaFirstGe + k] = first slot with B >= k (n if none), k = 1..kMaxOrder.
constexpr int kMetaFirstGe = 8;
constexpr int kMetaWords = kMetaFirstGe + kMaxOrder + 1;
hipError_t launch_store_meta(hipStream_t st, const uint8_t* B, int64_t n, const int64_t* batch_off, int64_t nb,
                             int64_t* meta);
// Exclusive prefix sum of n uint32 values in place; scratch holds
// scan_u32_scratch_words(n) words.
int64_t scan_u32_scratch_words(int64_t n);
hipError_t launch_scan_u32(hipStream_t st, uint32_t* a, int64_t n, uint32_t* scratch);
// The same for int64 values (scratch: scan_u32_scratch_words(n) int64 words).
hipError_t launch_scan_i64(hipStream_t st, int64_t* a, int64_t n, int64_t* scratch);

// ---- hot path (trace.hip)
// Where render tallies and reads: with img_tape (the render records the
// tape and one camera's FP64 image fits the LDS) the render kernel tallies
// nothing and the images are formed from the tape afterwards in FP64 LDS
// images; otherwise every contribution is an FP64 atomic on the output.
// grid_lds: the extinction grid is cached in LDS.
struct RenderPlan {
    bool grid_lds = false, img_tape = false;
    int n_wg = 1;
    int img_groups = 0;  // img_tape: image partials per camera
    size_t partial_bytes = 0;
};
RenderPlan plan_render(int fp64, int64_t nu, const DevCams& c, bool tape, int64_t n_slots, int64_t first_slot,
                       int n_cu);
// Whether the render prefix and the reweight form beta_t - beta_ref in LDS
// (then they need no prepared delta grid).
bool delta_grid_lds(int fp64, int64_t nu);
// Per-vertex prefix factors of the render, one task per (batch, b <= brender).
hipError_t launch_render_prefix(hipStream_t st, int fp64, const TraceArgs& a, const VertexLevels& lv, int n_cu);
// The persistent render kernel alone (its task counter a.work[0] must be zero,
// a.pbase filled by launch_render_prefix).
hipError_t launch_render(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const RenderPlan& p);
// Images from the tape (img_tape; nothing otherwise), divided by N Omega_p
// (scale = 1/N) like launch_render_finalize; partial holds p.partial_bytes.
hipError_t launch_render_reduce(hipStream_t st, const TraceArgs& a, const DevCams& c, const RenderPlan& p,
                                const void* partial, double scale, double* img);
hipError_t launch_render_finalize(hipStream_t st, double* img, const DevCams& c, double scale);
// rho = residual / (N Omega_p) (scale = 1/N); also sets *flag = 1 when flag is
// given and zeroes the first two counters of every line of the task-counter
// set work (the first gradient slab's).
hipError_t launch_grad_prep(hipStream_t st, const double* residual, double* rho, const DevCams& c, double scale,
                            int* flag, unsigned int* work);
// How the gradient is tallied: per-workgroup FP64 LDS partials of one slab of
// z layers at a time (reduced by a second kernel), when a layer fits the LDS
// budget and the grid needs few slabs, else FP64 atomics on the output.
struct GradPlan {
    bool lds = false;
    int slab_layers = 1, n_slabs = 1;
    int n_wg = 1;
    size_t partial_bytes = 0;
};
GradPlan plan_grad(int nx, int ny, int nz, int64_t n_slots, int64_t first_slot, int n_cu, bool tape);
// z layers [*z0, *z1) of slab i of a plan.
void grad_slab(const GradPlan& p, int nz, int i, int* z0, int* z1);
// Gradient weights from the tape (runs only when *a.tape_flag is 1).
hipError_t launch_grad_weights(hipStream_t st, const TraceArgs& a, const DevCams& c, const VertexLevels& lv, int n_cu);
// Gradient terms of slab i (z layers [i*slab_layers, min(nz, (i+1)*slab_layers))):
// the persistent grad kernels (task counters a.work[0] and a.work[1] must be
// zero): with a tape flag, the walk kernel on the stored weights and the
// recomputing kernel, exactly one of which does work; with lds,
// launch_grad_reduce then writes the slab's gradient.
// With walk_on_tape false and a tape flag given, only the recomputing kernel
// is launched (it works when the tape does not match).
hipError_t launch_grad(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const GradPlan& p, int slab,
                       void* partial, bool walk_on_tape = true);
// (also zeroes the task counters in work for the next slab's launch)
// (skipped, but for the counters, when skip is non-null and *skip is 1)
hipError_t launch_grad_reduce(hipStream_t st, const GradPlan& p, int nx, int ny, int nz, int slab,
                              const void* partial, double* grad, unsigned int* work, const int* skip = nullptr);
// Binned gradient on the tape (every kernel returns at once unless
// *a.tape_flag is 1): choose_grad_bins picks the slab axis (the one along
// which the connections to the cameras and the sun's rays move least) and the
// slab thickness; launch_grad_bin_init clears the task ranges and zeroes grad;
// after launch_grad_weights has set the ranges, launch_grad_bin_lists counts
// the tasks per slab, scans and lists them slab after slab;
// launch_grad_bin_walk cuts the lists into chunks and runs the persistent walk
// kernel (chunk counter at work[kBinChunkWord] zero at launch), which tallies
// a chunk's slab in LDS and writes it out as the chunk's partial; and
// launch_grad_bin_reduce adds each voxel's partials into grad.
GradBins choose_grad_bins(const DevScene& s, const DevCams& c, int64_t n_tasks);
// Whether one layer of the chosen axis fits the LDS and the slabs are few
// enough for the binning kernels' per-slab counters.
bool grad_bins_fit(const DevScene& s, const GradBins& g);
hipError_t launch_grad_bin_init(hipStream_t st, const TraceArgs& a, const GradBins& g);
hipError_t launch_grad_bin_lists(hipStream_t st, const TraceArgs& a, const GradBins& g, uint32_t* scan_scratch);
hipError_t launch_grad_bin_walk(hipStream_t st, const TraceArgs& a, const DevCams& c, const GradBins& g, int n_cu);
hipError_t launch_grad_bin_reduce(hipStream_t st, const TraceArgs& a, const GradBins& g);
// Bytes of g.partial for a walk launch on n_cu workgroups.
size_t grad_bin_partial_bytes(const DevScene& s, const GradBins& g, int n_cu);
// Per-workgroup sums of r and r^2 into a.partial[2*wg..]; *n_blocks workgroups.
hipError_t launch_reweight(hipStream_t st, int fp64, const TraceArgs& a, int n_cu, int64_t* n_blocks);
// Workgroups launch_reweight uses for a store of n_slots slots.
int64_t reweight_blocks(int64_t n_slots, int n_cu);
// flag = 0 if a[i] != b[i] bitwise for some i < n (flag set to 1 beforehand,
// by launch_grad_prep).
hipError_t launch_equal_flag(hipStream_t st, const float* a, const float* b, int64_t n, int* flag);

// ---- path-sorting ablation (ablation.hip)
// A per-path (CSR) copy of a store in one order: path q's records are
// rec[off[q] .. off[q+1]), its size B[q]; n paths.
struct TppView {
    const float4* rec;
    const int64_t* off;
    const uint8_t* B;
    int64_t n;
};
// Layout of the copy in `order` (0: the store's order, sorted by size; 1:
// path-id order, inv[id] = slot written from perm): off[0..n] = exclusive
// scan of the record counts (off[n] = total), qB = sizes; then the copy.
hipError_t launch_tpp_layout(hipStream_t st, const StoreView& sv, int64_t n, const int32_t* perm, int order,
                             int32_t* inv, int64_t* off, uint8_t* qB, void* scan_scratch);
hipError_t launch_tpp_copy(hipStream_t st, const StoreView& sv, int64_t n, const int32_t* inv, int order,
                           const int64_t* off, float4* rec);
// One thread per path: images (raw tallies, FP64 atomics on a.img) and the
// gradient terms of slab `slab` of plan p (LDS partials or FP64 atomics on
// a.grad, as the recomputing gradient kernel).
hipError_t launch_tpp_render(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const TppView& v,
                             int n_cu);
hipError_t launch_tpp_grad(hipStream_t st, int fp64, const TraceArgs& a, const DevCams& c, const TppView& v,
                           const GradPlan& p, int slab, double* partial);

// ---- loop glue (loop.hip)
hipError_t launch_fill(hipStream_t st, double* p, int64_t n, double v);
// loss = 0.5 sum (img - tgt)^2 and res = img - tgt.
hipError_t launch_loss(hipStream_t st, int64_t n, const double* img, const double* tgt, double* res,
                       double* partial, double* loss);
int64_t loss_blocks(int64_t n);
// out2[0] = sum of partial[2 i], out2[1] = sum of partial[2 i + 1] over
// i < n_blocks, in a fixed order (out2 may be pinned host memory).
hipError_t launch_sum_pairs(hipStream_t st, const double* partial, int64_t n_blocks, double* out2);
// stats[0] = (sum of partial[2i]) / n_paths, stats[1] = (sum partial[2i])^2 /
// sum partial[2i+1] (0 when that is 0), sums in launch_sum_pairs' order.
hipError_t launch_reweight_stats(hipStream_t st, const double* partial, int64_t n_blocks, double n_paths,
                                 double* stats);
struct CarveThresholds {
    double t[kMaxCams];
};
// mask[v] = 1 unless some camera sees the centre of voxel v on a pixel at or
// below its threshold; beta[v] (when given) = fill where kept, else 0.
hipError_t launch_space_carve(hipStream_t st, int nx, int ny, int nz, double vk, const DevCams& c,
                              const CarveThresholds& t, const double* img, float fill, uint8_t* mask, float* beta);
// coarse[d][R][C] = solid-angle-weighted mean of fine pixels
// (factor R + i, factor C + j), i, j < factor; c describes the fine cameras.
hipError_t launch_downsample(hipStream_t st, const DevCams& c, int factor, const double* fine, double* coarse);
// out[0] = epsilon, out[1] = delta of the estimate against the true field;
// partial holds 3 * volume_error_blocks(n) doubles.
int64_t volume_error_blocks(int64_t n);
hipError_t launch_volume_errors(hipStream_t st, int64_t n, const double* est, const float* truth, double* partial,
                                double* out);
hipError_t launch_adam(hipStream_t st, int64_t n, double* beta, float* beta_f32, const double* grad, double* m,
                       double* v, double lr, double b1, double b2, double eps, double bc1, double bc2);

}  // namespace prt
