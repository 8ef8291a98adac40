// Path sampling (Sec. 3.4), the stable counting sort by path size (Sec. 5.3)
// and the packing of the sorted paths into wavefront batches.
#include <algorithm>

#include "launch.hpp"

namespace prt {

// ------------------------------------------------------------- field prep

template <typename Real>
__global__ void __launch_bounds__(256) prep_grids_kernel(const float* __restrict__ bc_t,
                                                         const float* __restrict__ bc_r, double beta_air,
                                                         int64_t nu, Real* __restrict__ tot,
                                                         Real* __restrict__ dlt, float* __restrict__ copy,
                                                         unsigned int* __restrict__ zero, Real* __restrict__ tile,
                                                         int nx, int ny)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (zero && i == 0) *zero = 0u;
    if (i >= nu) return;
    const double t = (double)bc_t[i];
    if (tot) tot[i] = (Real)(t + beta_air);
    if (dlt) dlt[i] = (Real)(t - (double)bc_r[i]);
    if (copy) copy[i] = bc_t[i];
    if (tile) {
        const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
        tile[tile_index(ix, iy, iz, nx, ny)] = (Real)(t + beta_air);
    }
}

hipError_t launch_prep_grids(hipStream_t st, int fp64, const float* bc_t, const float* bc_r, double beta_air,
                             int64_t nu, void* grid_tot, void* grid_dlt, float* copy, unsigned int* zero, void* tile,
                             int nx, int ny)
{
    const int64_t blocks = (nu + 255) / 256;
    if (fp64)
        prep_grids_kernel<double><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(
            bc_t, bc_r, beta_air, nu, (double*)grid_tot, (double*)grid_dlt, copy, zero, (double*)tile, nx, ny);
    else
        prep_grids_kernel<float><<<dim3((unsigned)blocks), dim3(256), 0, st>>>(
            bc_t, bc_r, beta_air, nu, (float*)grid_tot, (float*)grid_dlt, copy, zero, (float*)tile, nx, ny);
    return hipGetLastError();
}

// ---------------------------------------------------------------- sampler

// Persistent sampler: one workgroup of kSampleBlock threads per CU holding the
// extinction grid in LDS when it fits kSampleLds, else kSampleBlocksPerCU
// workgroups per CU reading it from L2.
constexpr int kSampleBlock = 1024;
constexpr size_t kSampleLds = 128 * 1024;
constexpr int kSampleBlocksPerCU = 2;
// Free-flight pieces formed before their grid loads (grid in global memory).
// The all-FP64 walk keeps 4: it exceeds the 128 VGPRs of a lane of a
// 1024-thread workgroup either way, and workgroups of 512 threads without
// spills drew cloud32 in 1.21 ms against 1.04 ms.
template <typename Real>
constexpr int sample_loads()
{
    return sizeof(Real) == 8 ? 4 : 6;
}

// A uniform of (0,1) in the event precision, still below 1: in FP32 the
// largest uniforms round to 1.0f, which would give a free flight of zero
// optical depth (a scatter on top of the previous vertex).
template <typename E>
__device__ __forceinline__ E open_unit(double u);
template <>
__device__ __forceinline__ double open_unit<double>(double u) { return u; }
template <>
__device__ __forceinline__ float open_unit<float>(double u) { return fminf((float)u, 0x1.fffffep-1f); }

__device__ __forceinline__ float4 vrec(double x, double y, double z, int v)
{
    return make_float4((float)x, (float)y, (float)z, __int_as_float(v));
}

// Persistent sampler with path regeneration: a lane whose path has ended
// takes the next path id from its wavefront's pool of claimed ids, which is
// refilled 64 ids at a time from a device counter, so wavefronts do not wait
// for their longest path.  Each path is sampled as
// follows.  Entry point uniform over the projected box area; free flights by
// the DDA until the optical depth passes tau = -ln u; at a scatter the
// particle type is drawn with probability beta_s^(j)/beta_s and a direction
// from its phase function; the path ends when it leaves the box or after
// max_order scatters.  Vertices go where SampleArgs says (a row of tmp, the
// packed store, or nowhere).  The uniforms of path id come from its own
// Philox counters, so the result does not depend on which lane samples it.
template <typename Real, bool kGridLds>
__global__ void __launch_bounds__(kSampleBlock) sample_kernel(SampleArgs a)
{
    const DevScene& s = a.s;
    extern __shared__ unsigned char smem[];
    const Real* __restrict__ gt = (const Real*)a.grid_tot;
    if (kGridLds) {
        // the extinction grid in LDS: a piece's lookup waits ~100 clocks, not an L2 round trip
        Real* sg = reinterpret_cast<Real*>(smem);
        const int nu = s.nx * s.ny * s.nz;
        lds_fill(sg, nu, [&](int i) { return gt[i]; });
        __syncthreads();
        gt = sg;
    }
    const int stride = s.max_order + 2;
    const int lane = threadIdx.x % kWave;
    const uint64_t below = lane ? (~0ull >> (kWave - lane)) : 0ull;  // lanes under this one
    // short temporary rows: records from R on go to a chain of overflow
    // segments, taken from the wavefront's chunk [chunk[w][0], chunk[w][1])
    const bool compact = a.tmp && a.tmp_rows < stride;
    const int R = compact ? a.tmp_rows : stride;
    constexpr int kSegRec = kSegRecords - 1;  // records per segment
    __shared__ unsigned long long chunk[kSampleBlock / kWave][2];
    if (lane == 0) {
        chunk[threadIdx.x / kWave][0] = 0;
        chunk[threadIdx.x / kWave][1] = 0;
    }
    __syncthreads();
    int64_t oseg = -1;  // this path's current overflow segment (-2: none left)
    // path state and event arithmetic in the traversal precision
    using E = Real;
    int64_t id = 0;
    float4* __restrict__ out = nullptr;  // record k of the path at out[k * ostr]
    int64_t ostr = 1;
    E x = 0, y = 0, z = 0, tau = 0;
    E w[3] = {0, 0, 0};
    double u[4];
    int ix = 0, iy = 0, iz = 0, b = 0, nv = 0, v0 = 0;
    bool active = false, exhausted = false;
    // Ids claimed by this wavefront and not yet started: [pool, pool_end).
    // Claiming 64 at a time keeps the shared counter's atomics rare.
    int64_t pool = 0, pool_end = 0;
    for (;;) {
        uint64_t need = __ballot(!active);
        for (int round = 0; round < 2 && need && !exhausted; ++round) {
            if (pool == pool_end) {
                unsigned int base = 0;
                if (lane == 0) base = atomicAdd(a.next, (unsigned int)kWave);
                base = __shfl(base, 0);
                if ((int64_t)base >= a.n) {
                    exhausted = true;
                    break;
                }
                pool = base;
                pool_end = min((int64_t)base + kWave, a.n);
            }
            const int64_t take = min((int64_t)__popcll(need), pool_end - pool);
            const int64_t rank = __popcll(need & below);
            const int64_t nid = pool + rank;
            pool += take;
            if (!active && rank < take) {
                // start path nid at the source
                id = nid;
                oseg = -1;
                if (a.tmp) {
                    out = a.tmp + id * R;
                    ostr = 1;
                } else if (a.vtx) {
                    const int64_t sl = a.inv[id];
                    out = a.vtx + a.batch_off[sl / kWave] + sl % kWave;
                    ostr = kWave;
                } else {
                    out = nullptr;
                }
                uniforms4(a.seed, (uint64_t)id, 0u, u);
                const double A = s.a_top + s.a_x + s.a_y;
                if (u[0] * A < s.a_top) {
                    x = (E)(u[1] * s.nx); y = (E)(u[2] * s.ny); z = (E)s.nz;
                } else if (u[0] * A < s.a_top + s.a_x) {
                    x = (E)s.x_face; y = (E)(u[1] * s.ny); z = (E)(u[2] * s.nz);
                } else {
                    x = (E)(u[1] * s.nx); y = (E)s.y_face; z = (E)(u[2] * s.nz);
                }
                ix = min(max((int)floor(x), 0), s.nx - 1);
                iy = min(max((int)floor(y), 0), s.ny - 1);
                iz = min(max((int)floor(z), 0), s.nz - 1);
                nv = 0;
                v0 = ix + s.nx * (iy + s.ny * iz);
                if (out) out[nv * ostr] = vrec(x, y, z, v0);
                ++nv;
                w[0] = (E)s.sun[0]; w[1] = (E)s.sun[1]; w[2] = (E)s.sun[2];
                // optical depth target in units of (1/km * grid length)
                tau = -log(open_unit<E>(u[3])) / (E)s.vk;
                b = 0;
                active = true;
            }
            need = __ballot(!active);
        }
        if (!__any(active)) break;
        if (!active) continue;
        // one event: the free flight to the next scatter or out of the box
        const Real taur = (Real)tau;
        Real acc = (Real)0, thit = (Real)0, tend = (Real)0;
        int hit = -1;
        if constexpr (kGridLds) {
            tend = dda_walk<Real>(
                s.nx, s.ny, s.nz, (Real)x, (Real)y, (Real)z, ix, iy, iz, (Real)w[0], (Real)w[1], (Real)w[2],
                [&](int vv, Real t0, Real l) {
                    const Real dt = gt[vv] * l;  // zero for an empty voxel or a zero-length piece
                    if (taur < acc + dt) {
                        hit = vv;
                        thit = t0;
                        return false;
                    }
                    acc += dt;
                    return true;
                });
        } else {
            // the grid in global memory, z-tiled and walked in byte offsets:
            // sample_loads pieces per batch of loads; the hit's tiled index
            // becomes a linear one
            const unsigned char* __restrict__ gtl = (const unsigned char*)a.grid_tile;
            auto at = [&](uint32_t off) { return *reinterpret_cast<const Real*>(gtl + off); };
            const int ht = dda_first_hit<sample_loads<Real>(), Real, true, (int)sizeof(Real)>(
                s.nx, s.ny, s.nz, (Real)x, (Real)y, (Real)z, ix, iy, iz, (Real)w[0], (Real)w[1], (Real)w[2], taur, at,
                &acc, &thit);
            tend = thit;
            if (ht >= 0) {
                thit += (taur - acc) / at((uint32_t)ht);
                hit = tile_to_linear(ht / (int)sizeof(Real), s.nx, s.ny, s.inv_nx, s.inv_ny);
            }
        }
        // the division that places the scatter inside its voxel stays out of the loop
        if (kGridLds && hit >= 0) thit += (taur - acc) / gt[hit];
        // this event writes record nv: past the short row it goes to the
        // path's overflow segment, a new one taken now from the wavefront's
        // chunk when the current one is full
        if (compact) {
            const int j = nv - R;
            const bool need = j >= 0 && oseg != -2 && j % kSegRec == 0;
            const uint64_t m = __ballot(need);
            if (m) {
                // the first `old` lanes (in lane order) take the rest of the
                // chunk, the others the start of a new chunk claimed for them
                const int lead = __ffsll((unsigned long long)m) - 1;
                const unsigned long long cnt = (unsigned long long)__popcll(m);
                unsigned long long base = 0, old = 0, fresh = 0;
                if (lane == lead) {
                    const int w = threadIdx.x / kWave;
                    unsigned long long c0 = chunk[w][0], c1 = chunk[w][1];
                    base = c0;
                    old = min(cnt, c1 - c0);
                    c0 += old;
                    if (old < cnt) {
                        const unsigned long long take = max(cnt - old, (unsigned long long)a.ovf_chunk);
                        fresh = atomicAdd(a.ovf_next, take);
                        c0 = fresh + (cnt - old);
                        c1 = fresh + take;
                    }
                    chunk[w][0] = c0;
                    chunk[w][1] = c1;
                }
                base = __shfl(base, lead);
                old = __shfl(old, lead);
                fresh = __shfl(fresh, lead);
                if (need) {
                    const unsigned long long r = (unsigned long long)__popcll(m & below);
                    const unsigned long long blk = r < old ? base + r : fresh + (r - old);
                    if ((int64_t)blk < a.ovf_cap) {
                        if (j == 0)
                            a.ovf_slot[id] = (int32_t)blk;
                        else
                            a.ovf[oseg * kSegRecords + kSegRec] = make_float4(__int_as_float((int)blk), 0.f, 0.f, 0.f);
                        oseg = (int64_t)blk;
                    } else {
                        oseg = -2;
                        *a.ovf_full = 1;
                    }
                }
            }
        }
        // record k of the path: the short row, the overflow segment, the store
        auto put = [&](int k, float4 r) {
            if (k < R) {
                if (out) out[k * ostr] = r;
            } else if (oseg >= 0) {
                a.ovf[oseg * kSegRecords + (k - R) % kSegRec] = r;
            }
        };
        bool done;
        if (hit < 0) {
            put(nv, vrec(x + tend * w[0], y + tend * w[1], z + tend * w[2], -1));
            ++nv;
            done = true;
        } else {
            x = x + thit * w[0];
            y = y + thit * w[1];
            z = z + thit * w[2];
            ++b;
            put(nv, vrec(x, y, z, hit));
            ++nv;
            if (b == 1) v0 = hit;  // the sort key follows the first scatter
            done = b >= s.max_order;
            if (!done) {
                voxel_ijk(s, hit, ix, iy, iz);
                uniforms4(a.seed, (uint64_t)id, (uint32_t)b, u);
                // the particle choice is taken in FP64 in both precisions
                const double bsc = s.w_c * (double)a.beta_c[hit];
                const double bs = bsc + s.w_a * s.beta_air;
                const E mu = (u[0] * bs < bsc) ? sample_hg<E>((E)u[1], (E)s.g) : sample_rayleigh<E>((E)u[1]);
                E wn[3];
                scatter_direction<E>(w, mu, (E)(2.0 * kPi) * (E)u[2], wn);
                w[0] = wn[0]; w[1] = wn[1]; w[2] = wn[2];
                tau = -log(open_unit<E>(u[3])) / (E)s.vk;
            }
        }
        if (done) {
            if (a.vtx) {
                // second pass: the path must have the size the first pass found
                if (a.tB[id] != (uint8_t)b || a.tnv[id] != (uint8_t)nv) *a.mismatch = 1;
            } else {
                a.tB[id] = (uint8_t)b;
                a.tnv[id] = (uint8_t)nv;
                a.tC[id] = (uint16_t)cell_key(v0, s.nx, s.ny, s.nz);
            }
            active = false;
        }
    }
}

template <typename Real, bool kGridLds>
static hipError_t launch_sample_t(hipStream_t st, const SampleArgs& a, int64_t blocks, size_t lds)
{
    if (lds) {
        hipError_t e = hipFuncSetAttribute((const void*)sample_kernel<Real, kGridLds>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    sample_kernel<Real, kGridLds><<<dim3((unsigned)blocks), dim3(kSampleBlock), lds, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_sample(hipStream_t st, int fp64, const SampleArgs& a, int n_cu)
{
    if (a.n <= 0) return hipSuccess;
    const size_t lds = (size_t)a.s.nx * a.s.ny * a.s.nz * (fp64 ? 8 : 4);
    const bool grid_lds = lds <= kSampleLds;
    const int64_t blocks = std::min<int64_t>((a.n + kSampleBlock - 1) / kSampleBlock,
                                             (int64_t)n_cu * (grid_lds ? 1 : kSampleBlocksPerCU));
    if (fp64)
        return grid_lds ? launch_sample_t<double, true>(st, a, blocks, lds)
                        : launch_sample_t<double, false>(st, a, blocks, 0);
    return grid_lds ? launch_sample_t<float, true>(st, a, blocks, lds) : launch_sample_t<float, false>(st, a, blocks, 0);
}

// ----------------------------------------------------- stable counting sort

// Keys are processed in tiles of kSortTile positions; the key of position i
// is key[in[i]] (or key[i] without an input permutation).  Tile t's count of
// key k lives at hist[k * n_tiles + t], so an exclusive scan of hist in that
// order gives every (key, tile) its first output position.
constexpr int kSortTile = 4096;

// Optional outputs of a scatter pass: key_out[dst] = key of the element,
// aux_out[dst] = its aux byte for every sorted position dst, and zeros in
// [n, n_pad).
struct SortExtra {
    uint8_t* key_out = nullptr;
    uint8_t* aux_out = nullptr;
    int32_t* inv_out = nullptr;  // inv_out[element] = dst
    int64_t n_pad = 0;
};

// A key read: kPacked keys are the carried uint16 of position i (key in the
// low byte, aux in the high byte), so a pass over an earlier pass's output
// reads them in order instead of gathering key[in[i]].
template <typename K, bool kPacked>
__device__ __forceinline__ uint32_t sort_key_raw(const K* __restrict__ key, const int32_t* __restrict__ in, int64_t i)
{
    if constexpr (kPacked) return key[i];
    else return key[in ? in[i] : i];
}
constexpr int kMaxBins = kCells > kMaxOrder + 1 ? kCells : kMaxOrder + 1;

template <typename K, bool kPacked>
__global__ void __launch_bounds__(256) sort_hist_kernel(const K* __restrict__ key, const int32_t* __restrict__ in,
                                                        int64_t n, int nbins, int64_t n_tiles,
                                                        uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[kMaxBins];
    for (int i = threadIdx.x; i < nbins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = threadIdx.x; j < kSortTile; j += blockDim.x) {
        const int64_t i = base + j;
        if (i < n) {
            const uint32_t kr = sort_key_raw<K, kPacked>(key, in, i);
            atomicAdd(&h[min((int)(kPacked ? kr & 0xffu : kr), nbins - 1)], 1u);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nbins; k += blockDim.x) hist[(int64_t)k * n_tiles + blockIdx.x] = h[k];
}

// Exclusive prefix sum in place, tiled: each workgroup scans a tile of
// kScanTile values (4 consecutive values per thread, a Hillis-Steele scan of
// the 256 thread totals in LDS) and writes the tile total; the tile totals
// are scanned the same way (recursively) and added back to their tiles.
constexpr int kScanTile = 1024;

template <typename T>
__global__ void __launch_bounds__(256) scan_tile_kernel(T* __restrict__ a, int64_t n, T* __restrict__ tile_sum)
{
    __shared__ T s[256];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + 4 * t;
    T e[4];
    T run = 0;
    for (int k = 0; k < 4; ++k) {
        const T v = i0 + k < n ? a[i0 + k] : (T)0;
        e[k] = run;
        run += v;
    }
    s[t] = run;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const T add = t >= off ? s[t - off] : (T)0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    const T before = t ? s[t - 1] : (T)0;
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n) a[i0 + k] = before + e[k];
    if (t == 255 && tile_sum) tile_sum[blockIdx.x] = s[255];
}

template <typename T>
__global__ void __launch_bounds__(256) scan_add_kernel(T* __restrict__ a, int64_t n, const T* __restrict__ tile_off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += tile_off[i / kScanTile];
}

// Elements of scratch that scan_exclusive needs for n values.
static int64_t scan_scratch_elems(int64_t n)
{
    int64_t tot = 0;
    for (int64_t m = n; m > kScanTile;) {
        m = (m + kScanTile - 1) / kScanTile;
        tot += m;
    }
    return tot;
}

template <typename T>
static hipError_t scan_exclusive(hipStream_t st, T* a, int64_t n, T* scratch)
{
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        scan_tile_kernel<T><<<dim3(1), dim3(256), 0, st>>>(a, n, nullptr);
        return hipGetLastError();
    }
    scan_tile_kernel<T><<<dim3((unsigned)tiles), dim3(256), 0, st>>>(a, n, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = scan_exclusive<T>(st, scratch, tiles, scratch + tiles)) != hipSuccess) return e;
    scan_add_kernel<T><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>(a, n, scratch);
    return hipGetLastError();
}

// One wavefront per tile, which takes the tile 64 positions at a time in
// position order: each lane finds the lanes holding its key (one ballot per
// key bit), counts those below it, so equal keys keep their order, and the
// last lane of each key advances that key's running output position in LDS.
// Writes out[pos] = in[i] (or i).
template <typename K, bool kPacked>
__global__ void __launch_bounds__(kWave) sort_scatter_kernel(const K* __restrict__ key,
                                                             const int32_t* __restrict__ in, int64_t n, int nbins,
                                                             int64_t n_tiles, const uint32_t* __restrict__ off,
                                                             int32_t* __restrict__ out, SortExtra x)
{
    if (x.key_out && blockIdx.x == 0)
        for (int64_t i = n + threadIdx.x; i < x.n_pad; i += kWave) {
            x.key_out[i] = 0;
            x.aux_out[i] = 0;
        }
    __shared__ uint32_t base[kMaxBins];
    for (int k = threadIdx.x; k < nbins; k += kWave) base[k] = off[(int64_t)k * n_tiles + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x;
    const uint64_t below_mask = lane ? (~0ull >> (kWave - lane)) : 0ull;
    int nbits = 1;
    while ((1 << nbits) < nbins) ++nbits;
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortTile / kWave; ++r) {
        const int64_t i = t0 + r * kWave + lane;
        const bool valid = i < n;
        const uint32_t kr = valid ? sort_key_raw<K, kPacked>(key, in, i) : 0u;
        const int k = min((int)(kPacked ? kr & 0xffu : kr), nbins - 1);
        uint64_t same = __ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool set = (k >> bit) & 1;
            const uint64_t bb = __ballot(set);
            same &= set ? bb : ~bb;
        }
        if (valid) {
            const int below = __popcll(same & below_mask), total = __popcll(same);
            const int32_t id = in ? in[i] : (int32_t)i;
            const uint32_t dst = base[k] + below;
            out[dst] = id;
            if (x.key_out) {
                x.key_out[dst] = (uint8_t)kr;
                x.aux_out[dst] = (uint8_t)(kr >> 8);
            }
            if (x.inv_out) x.inv_out[id] = (int32_t)dst;
            if (below == total - 1) base[k] += total;
        }
        __syncthreads();
    }
}

// The cell pass, staged through LDS.  The wavefront loads its tile's keys
// and carried bytes into LDS, ranks every key within the tile with the same
// ballots as sort_scatter_kernel (equal keys keep their order), records
// which element lands at each local position, and then writes the tile out in
// local order: consecutive lanes write consecutive positions of one key's run
// (4096 keys over 512 cells, runs of 8 on average) instead of one line per
// lane.  Writes out[dst] = i and carry_out[dst] = carry_lo[i] |
// carry_hi[i] << 8, which carries two bytes of every element into cell order.
__global__ void __launch_bounds__(kWave) sort_scatter_cells_kernel(
    const uint16_t* __restrict__ key, int64_t n, int64_t n_tiles, const uint32_t* __restrict__ off,
    int32_t* __restrict__ out, const uint8_t* __restrict__ carry_lo, const uint8_t* __restrict__ carry_hi,
    uint16_t* __restrict__ carry_out)
{
    constexpr int kPer = kCells / kWave;
    static_assert(kPer * kWave == kCells && kSortTile <= 65536, "cell pass layout");
    __shared__ uint32_t gbase[kCells];   // first output position of key k for this tile
    __shared__ uint32_t lstart[kCells];  // first local position of key k
    __shared__ uint32_t lrun[kCells];    // next free local position of key k
    __shared__ uint16_t kin[kSortTile];  // the tile's keys
    __shared__ uint16_t cin[kSortTile];  // the tile's carried bytes
    __shared__ uint16_t src[kSortTile];  // tile offset of the element at each local position
    const int lane = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * kSortTile;
    const int cnt = (int)min<int64_t>(kSortTile, n - t0);
    for (int j = lane; j < cnt; j += kWave) {
        kin[j] = (uint16_t)min((int)key[t0 + j], kCells - 1);
        cin[j] = (uint16_t)(carry_lo[t0 + j] | (uint32_t)carry_hi[t0 + j] << 8);
    }
    // this tile's count of key k: the entry after (k, tile) in scan order is
    // (k, tile + 1), or (k + 1, 0) for the last tile; n follows the last entry
    const int64_t m = (int64_t)kCells * n_tiles;
    uint32_t c[kPer], tot = 0;
    for (int q = 0; q < kPer; ++q) {
        const int k = lane * kPer + q;
        const int64_t idx = (int64_t)k * n_tiles + blockIdx.x;
        const uint32_t g = off[idx];
        c[q] = (idx + 1 < m ? off[idx + 1] : (uint32_t)n) - g;
        gbase[k] = g;
        tot += c[q];
    }
    uint32_t incl = tot;
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    uint32_t run = incl - tot;
    for (int q = 0; q < kPer; ++q) {
        lstart[lane * kPer + q] = run;
        lrun[lane * kPer + q] = run;
        run += c[q];
    }
    __syncthreads();
    const uint64_t below_mask = lane ? (~0ull >> (kWave - lane)) : 0ull;
    for (int r = 0; r * kWave < cnt; ++r) {
        const int j = r * kWave + lane;
        const bool valid = j < cnt;
        const int k = valid ? (int)kin[j] : 0;
        uint64_t same = __ballot(valid);
        for (int bit = 0; bit < 3 * kCellBits; ++bit) {
            const bool set = (k >> bit) & 1;
            const uint64_t bb = __ballot(set);
            same &= set ? bb : ~bb;
        }
        if (valid) {
            const int below = __popcll(same & below_mask), total = __popcll(same);
            src[lrun[k] + below] = (uint16_t)j;
            if (below == total - 1) lrun[k] += total;
        }
        __syncthreads();
    }
    for (int j = lane; j < cnt; j += kWave) {
        const int e = src[j];
        const int k = kin[e];
        const uint32_t dst = gbase[k] + (uint32_t)(j - (int)lstart[k]);
        out[dst] = (int32_t)(t0 + e);
        carry_out[dst] = cin[e];
    }
}

int64_t scan_u32_scratch_words(int64_t n) { return scan_scratch_elems(n); }

hipError_t launch_scan_i64(hipStream_t st, int64_t* a, int64_t n, int64_t* scratch)
{
    return scan_exclusive<int64_t>(st, a, n, scratch);
}

hipError_t launch_scan_u32(hipStream_t st, uint32_t* a, int64_t n, uint32_t* scratch)
{
    return scan_exclusive<uint32_t>(st, a, n, scratch);
}

template <typename K, bool kPacked = false>
static hipError_t counting_sort(hipStream_t st, const K* key, const int32_t* in, int64_t n, int nbins,
                                uint32_t* hist, int32_t* out, SortExtra x = SortExtra{})
{
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    sort_hist_kernel<K, kPacked><<<dim3((unsigned)n_tiles), dim3(256), 0, st>>>(key, in, n, nbins, n_tiles, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t m = n_tiles * nbins;
    if ((e = scan_exclusive<uint32_t>(st, hist, m, hist + m)) != hipSuccess) return e;
    sort_scatter_kernel<K, kPacked><<<dim3((unsigned)n_tiles), dim3(kWave), 0, st>>>(key, in, n, nbins, n_tiles,
                                                                                     hist, out, x);
    return hipGetLastError();
}

int64_t sort_scratch_words(int64_t n, int nbins)
{
    const int64_t tiles = (n + kSortTile - 1) / kSortTile;
    const int64_t hist = tiles * (int64_t)std::max(nbins, kCells);
    const int64_t sort_words = hist + scan_scratch_elems(hist);
    // launch_batch_offsets reuses the same scratch for its int64 scan
    const int64_t nb = (n + kWave - 1) / kWave;
    const int64_t boff_words = 2 * scan_scratch_elems(nb + 1);
    return std::max<int64_t>(1, std::max(sort_words, boff_words));
}

hipError_t launch_sort_paths(hipStream_t st, const uint8_t* size_key, const uint8_t* tnv, const uint16_t* cell,
                             int64_t n, int64_t n_slots, int nbins, uint32_t* hist, int32_t* tmp_perm,
                             uint16_t* carry, int32_t* perm, uint8_t* B, uint8_t* nv, int32_t* inv)
{
    if (n <= 0) return hipSuccess;
    // the cell pass carries every path's size key and vertex count along,
    // so the size pass reads them in order
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    sort_hist_kernel<uint16_t, false><<<dim3((unsigned)n_tiles), dim3(256), 0, st>>>(cell, nullptr, n, kCells,
                                                                                     n_tiles, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = scan_exclusive<uint32_t>(st, hist, n_tiles * kCells, hist + n_tiles * kCells)) != hipSuccess) return e;
    sort_scatter_cells_kernel<<<dim3((unsigned)n_tiles), dim3(kWave), 0, st>>>(cell, n, n_tiles, hist, tmp_perm,
                                                                               size_key, tnv, carry);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the size pass also writes every slot's B and vertex count (zero past n)
    SortExtra x;
    x.key_out = B;
    x.aux_out = nv;
    x.inv_out = inv;
    x.n_pad = n_slots;
    return counting_sort<uint16_t, true>(st, carry, tmp_perm, n, nbins, hist, perm, x);
}

// --------------------------------------------------------------- packing

// batch_off[b] = 64 * sum_{b' < b} rows(b'), rows(b) = max stored vertices
// over the batch; batch_off[nb] is the total record count.  One wavefront
// per batch writes 64 * rows(b) (and batch_off[nb] = 0), then an exclusive
// scan turns the counts into offsets.
__global__ void __launch_bounds__(256) batch_rows_kernel(const uint8_t* __restrict__ nv, int64_t nb,
                                                         int64_t* __restrict__ off)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = i / kWave;
    int r = b < nb ? (int)nv[i] : 0;
    for (int o = kWave / 2; o > 0; o >>= 1) r = max(r, __shfl_xor(r, o));
    if (i % kWave == 0 && b < nb) off[b] = (int64_t)r * kWave;
    if (i == 0) off[nb] = 0;
}

hipError_t launch_batch_offsets(hipStream_t st, const uint8_t* nv, int64_t nb, int64_t* batch_off, void* scratch)
{
    const int64_t slots = nb * kWave;
    batch_rows_kernel<<<dim3((unsigned)std::max<int64_t>(1, (slots + 255) / 256)), dim3(256), 0, st>>>(nv, nb,
                                                                                                     batch_off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return scan_exclusive<int64_t>(st, batch_off, nb + 1, (int64_t*)scratch);
}

// One thread per sorted slot: copy the path's records into its lane of the
// batch (rows beyond its own vertex count are zero-filled).
constexpr int kPackLoads = 4;

__global__ void __launch_bounds__(256) pack_kernel(const int32_t* __restrict__ perm, const float4* __restrict__ tmp,
                                                   const int64_t* __restrict__ tmp_off, int64_t tmp_stride,
                                                   const uint8_t* __restrict__ nv,
                                                   const int64_t* __restrict__ batch_off, int64_t n,
                                                   int64_t n_slots, float4* __restrict__ vtx,
                                                   const float4* __restrict__ ovf, const int32_t* __restrict__ ovf_slot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_slots) return;
    const int64_t b = i / kWave, lane = i % kWave;
    const int64_t rows = (batch_off[b + 1] - batch_off[b]) / kWave;
    float4* dst = vtx + batch_off[b] + lane;
    const int cnt = i < n ? (int)nv[i] : 0;
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4* src = nullptr;
    int64_t id = 0;
    if (i < n) {
        id = perm[i];
        src = tmp + (tmp_off ? tmp_off[id] : id * tmp_stride);
    }
    if (!ovf) {
        // whole rows: kPackLoads records of the path in flight at a time
        for (int64_t k0 = 0; k0 < rows; k0 += kPackLoads) {
            float4 r[kPackLoads];
#pragma unroll
            for (int j = 0; j < kPackLoads; ++j) {
                const int64_t k = k0 + j;
                r[j] = k < cnt ? src[k] : zero;
            }
#pragma unroll
            for (int j = 0; j < kPackLoads; ++j)
                if (k0 + j < rows) dst[(k0 + j) * kWave] = r[j];
        }
        return;
    }
    // short row, then one overflow segment at a time (its records and its
    // link in flight together)
    for (int64_t k = 0; k < tmp_stride && k < rows; ++k) dst[k * kWave] = k < cnt ? src[k] : zero;
    constexpr int kSegRec = kSegRecords - 1;
    const float4* seg = cnt > tmp_stride ? ovf + (int64_t)ovf_slot[id] * kSegRecords : nullptr;
    for (int64_t k0 = tmp_stride; k0 < rows; k0 += kSegRec) {
        float4 r[kSegRecords];
#pragma unroll
        for (int j = 0; j < kSegRecords; ++j) r[j] = seg && k0 + j < cnt ? seg[j] : zero;
#pragma unroll
        for (int j = 0; j < kSegRec; ++j)
            if (k0 + j < rows) dst[(k0 + j) * kWave] = r[j];
        // the link is set when the path has a record past this segment
        seg = seg && k0 + kSegRec < cnt ? ovf + (int64_t)__float_as_int(r[kSegRec].x) * kSegRecords : nullptr;
    }
}

hipError_t launch_pack(hipStream_t st, const int32_t* perm, const float4* tmp, const int64_t* tmp_off,
                       int64_t tmp_stride, const uint8_t* nv, const int64_t* batch_off, int64_t n, int64_t n_slots,
                       float4* vtx, const float4* ovf, const int32_t* ovf_slot)
{
    pack_kernel<<<dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st>>>(
        perm, tmp, tmp_off, tmp_stride, nv, batch_off, n, n_slots, vtx, ovf, ovf_slot);
    return hipGetLastError();
}

// Store metadata read back once after packing (see launch.hpp).
__global__ void store_meta_kernel(const uint8_t* __restrict__ B, int64_t n, const int64_t* __restrict__ batch_off,
                                  int64_t nb, int64_t* __restrict__ meta)
{
    // slots are sorted by B: thread k-1 binary-searches the first slot with B >= k
    const int k = (int)threadIdx.x + 1;
    if (blockIdx.x != 0 || k > kMaxOrder) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if ((int)B[mid] >= k) hi = mid; else lo = mid + 1;
    }
    meta[kMetaFirstGe + k] = lo;
    if (k == 1) {
        meta[0] = batch_off[nb];
        meta[1] = lo;
        meta[2] = lo < n ? batch_off[lo / kWave] : batch_off[nb];
    }
}

hipError_t launch_store_meta(hipStream_t st, const uint8_t* B, int64_t n, const int64_t* batch_off, int64_t nb,
                             int64_t* meta)
{
    store_meta_kernel<<<dim3(1), dim3(kMaxOrder), 0, st>>>(B, n, batch_off, nb, meta);
    return hipGetLastError();
}

}  // namespace prt
