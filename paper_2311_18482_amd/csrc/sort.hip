// Tile binning for the rasteriser (gfx950): per-tile lists of (tile << 32 |
// depth bits) keys and Gaussian ids, each list in depth order (ties by
// Gaussian), and per-tile [start, end) ranges.
//
// Depth-first path (default): the G-views are sorted once by (view, depth
// bits) with a stable LSD onesweep radix sort; each G-view's rectangle of
// 8 x 4-tile super-tiles is written out in that order and sorted stably by
// super-tile id (reduce-then-scan counting passes); a compaction then splits
// each super-tile's list into its 32 tile lists, writing every instance once,
// at its final place. Per-cell counts of both streams come from 2D difference
// grids over the rectangles, so ranges and offsets are known without reading
// any instance. Full-sort path (LEGS_FLAG_FULL_SORT): every instance is
// emitted in Gaussian order and all key digits are sorted over the instances.
//
// Every kernel after the scan reads its sizes from device memory and walks
// them with a fixed grid, so the whole chain can be captured in a HIP graph
// without knowing the counts on the host.
//
// Onesweep (one pass per digit of up to 8 bits): each pass ranks a 4096-key
// partition per workgroup with wave64 ballots (stable: ties keep input order),
// scatters the keys into LDS in digit order, and writes them out so that
// consecutive lanes write consecutive addresses within a digit run. Global
// digit offsets come either from a decoupled look-back over earlier
// partitions (partition ids handed out by an atomic counter in launch order,
// so every partition waited on belongs to a running workgroup) or, for the
// segment passes, from per-segment digit counts scanned beforehand.
#include "legs_internal.h"

namespace {

constexpr uint64_t FLAG_AGG = 1ull << 62;
constexpr uint64_t FLAG_INC = 2ull << 62;
constexpr uint64_t VALUE_MASK = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t ld_status(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- scan of the per-block instance counts -----------------------------------

// Inclusive sum over lanes 0..l of a wave (DPP row shifts, then the row
// broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t x)
{
#define LEGS_DPP_ADD(ctrl, rmask) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, ctrl, rmask, 0xF, false);
    LEGS_DPP_ADD(0x111, 0xF)   // row_shr:1
    LEGS_DPP_ADD(0x112, 0xF)   // row_shr:2
    LEGS_DPP_ADD(0x114, 0xF)   // row_shr:4
    LEGS_DPP_ADD(0x118, 0xF)   // row_shr:8
    LEGS_DPP_ADD(0x142, 0xA)   // row_bcast:15 into rows 1 and 3
    LEGS_DPP_ADD(0x143, 0xC)   // row_bcast:31 into rows 2 and 3
#undef LEGS_DPP_ADD
    return x;
}

__device__ __forceinline__ uint64_t wave_incl_add(uint64_t x)
{
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint64_t y = __shfl_up(x, off, LEGS_WAVE);
        if (legs_lane() >= off) x += y;
    }
    return x;
}

// One workgroup of 1024 threads: exclusive scan of x(i), i in [0, n), handed
// to emit(i, exclusive prefix, x(i)); returns the total. A round covers ROWS *
// 1024 values: wave w scans its ROWS * 64 consecutive values as ROWS coalesced
// rows (all loads in flight together), then adds the sums of the waves before
// it. ROWS keeps the 64-bit scan within the 128 registers a 1024-thread
// workgroup allows; the 32-bit scans (tile and unit counts, a few thousand
// to tens of thousands) take shorter rounds.
template <typename T, typename X, typename E, int ROWS = sizeof(T) == 8 ? 8 : 4>
__device__ __forceinline__ T scan_rounds(int64_t n, X x, E emit)
{
    constexpr int NW = 1024 / LEGS_WAVE;
    __shared__ T s_w[NW];
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    T carry = 0;
    for (int64_t base = 0; base < n; base += (int64_t)ROWS * 1024) {
        const int64_t w0 = base + (int64_t)wave * ROWS * LEGS_WAVE + lane;
        T v[ROWS], e[ROWS];
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const int64_t i = w0 + j * LEGS_WAVE;
            v[j] = i < n ? x(i) : (T)0;
        }
        T run = 0;
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const T incl = wave_incl_add(v[j]);
            const T row = __shfl(incl, LEGS_WAVE - 1, LEGS_WAVE);
            e[j] = run + incl - v[j];
            run += row;
        }
        if (lane == 0) s_w[wave] = run;
        __syncthreads();
        T pre = carry, all = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const T t = s_w[w];
            pre += w < wave ? t : (T)0;
            all += t;
        }
#pragma unroll
        for (int j = 0; j < ROWS; ++j) {
            const int64_t i = w0 + j * LEGS_WAVE;
            if (i < n) emit(i, pre + e[j], v[j]);
        }
        carry += all;
        __syncthreads();
    }
    return carry;
}

// One workgroup: exclusive scan of counts[0..nb) into offsets[0..nb], total
// in offsets[nb] and in *total (counts stay intact, so the binning can rerun).
__device__ __forceinline__ void scan_blocks(const uint64_t *__restrict__ counts, uint64_t *__restrict__ offsets,
                                            int64_t nb, uint64_t *__restrict__ total)
{
    const uint64_t t = scan_rounds<uint64_t>(
        nb, [&](int64_t i) { return counts[i]; }, [&](int64_t i, uint64_t e, uint64_t) { offsets[i] = e; });
    if (threadIdx.x == 0) {
        offsets[nb] = t;
        *total = t;
    }
}

__global__ void __launch_bounds__(1024)
k_scan_blocks(const uint64_t *__restrict__ counts, uint64_t *__restrict__ offsets, int64_t nb,
              uint64_t *__restrict__ total)
{
    scan_blocks(counts, offsets, nb, total);
}

// Two independent scans, one workgroup each.
struct ScanArgs {
    const uint64_t *counts;
    uint64_t *offsets;
    int64_t nb;
    uint64_t *total;
};

__global__ void __launch_bounds__(1024) k_scan_pair(ScanArgs a, ScanArgs b)
{
    const ScanArgs &x = blockIdx.x == 0 ? a : b;
    scan_blocks(x.counts, x.offsets, x.nb, x.total);
}

// ---- emission -------------------------------------------------------------------

// Same grid as the projection: block (bx, v) owns G-views [v n + 256 bx, ...).
// The block's instances are laid out Gaussian-major, tiles row-major inside
// each rectangle; threads stride over them (balanced even when one Gaussian
// covers thousands of tiles) and find their owner by binary search in LDS.
__global__ void __launch_bounds__(LEGS_PROJ_BLOCK)
k_emit(const int4 *__restrict__ box, const float *__restrict__ depth,
       const uint32_t *__restrict__ ntiles, const uint64_t *__restrict__ block_offsets, int64_t n,
       const legs_view *__restrict__ views, int tile, int64_t capacity,
       uint64_t *__restrict__ keys, uint32_t *__restrict__ ids)
{
    __shared__ uint32_t s_start[LEGS_PROJ_BLOCK + 1];
    __shared__ int s_tx0[LEGS_PROJ_BLOCK], s_ty0[LEGS_PROJ_BLOCK], s_rw[LEGS_PROJ_BLOCK];
    __shared__ uint32_t s_bits[LEGS_PROJ_BLOCK];
    const int v = blockIdx.y;
    const int64_t g = (int64_t)blockIdx.x * LEGS_PROJ_BLOCK + threadIdx.x;
    const int64_t gv = (int64_t)v * n + g;
    uint32_t cnt = 0;
    if (g < n) {
        cnt = ntiles[gv];
        if (cnt) {
            const int4 b = box[gv];
            s_tx0[threadIdx.x] = b.x / tile;
            s_ty0[threadIdx.x] = b.z / tile;
            s_rw[threadIdx.x] = b.y / tile - b.x / tile + 1;
            s_bits[threadIdx.x] = __float_as_uint(depth[gv]);
        }
    }
    // block-exclusive scan of cnt
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    __shared__ uint32_t s_w[LEGS_PROJ_BLOCK / LEGS_WAVE];
    if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += s_w[w];
    s_start[threadIdx.x] = wpre + incl - cnt;
    if (threadIdx.x == LEGS_PROJ_BLOCK - 1) s_start[LEGS_PROJ_BLOCK] = wpre + incl;
    __syncthreads();
    const uint32_t total = s_start[LEGS_PROJ_BLOCK];
    const uint64_t base = block_offsets[(int64_t)v * gridDim.x + blockIdx.x];
    const legs_view vw = views[v];
    for (uint32_t k = threadIdx.x; k < total; k += LEGS_PROJ_BLOCK) {
        // owner: last o with s_start[o] <= k
        int lo = 0, hi = LEGS_PROJ_BLOCK - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= k) lo = mid; else hi = mid - 1;
        }
        const uint32_t local = k - s_start[lo];
        const int rw = s_rw[lo];
        const int ty = s_ty0[lo] + (int)(local / (uint32_t)rw);
        const int tx = s_tx0[lo] + (int)(local % (uint32_t)rw);
        const uint64_t gt = (uint64_t)(vw.tile_offset + (int64_t)ty * vw.tiles_x + tx);
        const uint64_t pos = base + k;
        if (pos < (uint64_t)capacity) {
            keys[pos] = (gt << 32) | s_bits[lo];
            ids[pos] = (uint32_t)((int64_t)blockIdx.x * LEGS_PROJ_BLOCK + lo);
        }
    }
}

// ---- digit histograms for every pass in one read -----------------------------

constexpr int HIST_RUN = 16;  // keys per lane per block iteration

// Adds each valid lane's digit to an LDS histogram: the lanes holding the
// first valid lane's digit add with one atomic, the others with one each, so
// a wave of equal digits (the high digits of clustered keys) does not
// serialise on one LDS address. Called by every lane of the wave.
__device__ __forceinline__ void hist_add(uint32_t *h, uint32_t d, bool ok)
{
    const uint64_t valid = legs_ballot(ok);
    if (valid == 0) return;
    const int lead = __builtin_ctzll(valid);
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, lead);
    const uint64_t same = legs_ballot(ok && d == d0);
    if (ok && d != d0) atomicAdd(&h[d], 1u);
    if (legs_lane() == lead) atomicAdd(&h[d0], (uint32_t)__popcll(same));
}

// Digit histograms of passes [first, first + npass) in one read of the
// instance keys. Loads are coalesced (lane l reads key base + 64 i + l).
// Within each wave a run of equal digits in consecutive lanes is counted with
// one LDS atomic by its first lane (run starts from a ballot); instance keys
// come in long runs (every tile of one Gaussian shares its depth digits,
// consecutive tiles of a row share the high tile digits), so hot digits do not
// serialise. (The G-view depth keys are counted where they are made, in
// k_order_keys.)
__global__ void __launch_bounds__(256)
k_histogram(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ count,
            int64_t capacity, int first, int npass, uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_h[LEGS_SORT_MAX_PASSES][256];
    for (int i = threadIdx.x; i < LEGS_SORT_MAX_PASSES * 256; i += 256) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    const uint64_t above = lane == 63 ? 0ull : (~0ull << (lane + 1));
    const int64_t chunk = (int64_t)256 * HIST_RUN;
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < m; base += (int64_t)gridDim.x * chunk) {
        const int64_t wbase = base + (int64_t)wave * LEGS_WAVE * HIST_RUN;
        for (int i = 0; i < HIST_RUN; ++i) {
            const int64_t idx = wbase + (int64_t)i * LEGS_WAVE + lane;
            const bool ok = idx < m;
            const uint64_t k = ok ? keys[idx] : 0ull;
            for (int p = 0; p < npass; ++p) {
                const uint32_t d = ok ? ((uint32_t)(k >> (8 * (first + p))) & 255u) : 256u;
                const uint32_t dp = (uint32_t)__shfl_up((int)d, 1, LEGS_WAVE);
                const uint64_t starts = legs_ballot(lane == 0 || d != dp);
                if (ok && (lane == 0 || d != dp)) {
                    const uint64_t nxt = starts & above;
                    const int end = nxt ? __ffsll((unsigned long long)nxt) - 1 : LEGS_WAVE;
                    atomicAdd(&s_h[p][d], (uint32_t)(end - lane));
                }
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += 256) {
        const uint32_t c = (&s_h[0][0])[i];
        if (c) atomicAdd(&hist[(first + i / 256) * 256 + (i % 256)], c);
    }
}

// Zero the look-back status words of every pass and the partition counters,
// only as far as the partitions this count needs.
struct SortClearArgs {
    uint64_t *status;
    int64_t parts_cap;
    int passes;
    uint32_t *counters, *hist;
    const uint64_t *count;   // NULL: the count is not known yet (capacity is used)
    int64_t capacity;
};

// The share of workgroup `block` of `blocks`.
__device__ __forceinline__ void sort_clear_part(const SortClearArgs &a, int64_t block, int64_t blocks)
{
    if (a.passes <= 0) return;
    const uint64_t cnt = a.count ? *a.count : (uint64_t)a.capacity;
    const int64_t m = (int64_t)(cnt < (uint64_t)a.capacity ? cnt : (uint64_t)a.capacity);
    const int64_t parts = (m + LEGS_SORT_PART - 1) / LEGS_SORT_PART;
    const int64_t per_pass = parts * 256;
    const int64_t tot = per_pass * a.passes;
    const int64_t stride = blocks * 256;
    for (int64_t i = block * 256 + threadIdx.x; i < tot; i += stride) {
        const int64_t p = i / per_pass, r = i - p * per_pass;
        a.status[p * a.parts_cap * 256 + r] = 0;
    }
    if (block == 0 && a.counters) {
        if (threadIdx.x < 16) a.counters[threadIdx.x] = 0;
        for (int i = threadIdx.x; i < LEGS_SORT_MAX_PASSES * 256; i += 256) a.hist[i] = 0;
    }
}

__global__ void __launch_bounds__(256) k_sort_clear(SortClearArgs a)
{
    sort_clear_part(a, blockIdx.x, gridDim.x);
}

// Super-tile record of a depth-ordered position: what the coarse pass needs
// of the G-view there, read once with one coalesced load.
struct GRec {
    uint32_t gid;    // the position itself (the coarse lists hold positions)
    uint32_t cnt;    // super-tiles of its rectangle (0: culled)
    uint32_t base;   // global id of its first super-tile
    uint32_t rwtx;   // rectangle width | super-tiles per row of its view << 16
};

// Tile record of a depth-ordered position: its tile rectangle in view-local
// tile coordinates (the per-tile counts and the compaction read it).
struct FRec {
    uint32_t gid;    // Gaussian index
    uint32_t dbits;  // depth bits
    uint32_t xy;     // first tile column | first tile row << 16
    uint32_t wh;     // rectangle width | height << 16 (0: culled)
};

// The tile records the last coarse pass carries out with the sorted list:
// pay[i] = frecs[position of list entry i] (positions >= G give zeros).
struct CoarsePay {
    const FRec *frecs;
    FRec *pay;
    int64_t G;
};

// Exclusive scan over a block of T threads of one 64-bit value per thread
// (threads >= 256 pass 0); s_start[0..256] receives the scan of the first
// 256 and their total.
template <int T>
__device__ __forceinline__ void block_scan_256(uint64_t x, uint64_t *s_start, uint64_t *s_w)
{
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    uint64_t incl = x;
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint64_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
    __syncthreads();
    if (threadIdx.x < 256) {
        uint64_t wpre = 0;
        for (int w = 0; w < wave; ++w) wpre += s_w[w];
        s_start[threadIdx.x] = wpre + incl - x;
        if (threadIdx.x == 255) s_start[256] = wpre + incl;
    }
    __syncthreads();
}

// Digit layout of the coarse passes, decided on the device from the number of
// super-tiles: desc[0] passes, desc[2 + 2p] and desc[3 + 2p] the shift and
// width of pass p (width 0: the pass is not needed and returns at once).

// One onesweep pass over the digit of `rb` bits at `shift` of keys K with
// 32-bit values (with desc, shift and width come from desc[2 + 2 pass ..]).
// SEG: workgroups walk fixed segments of partitions in order from the segment
// digit starts instead of a decoupled look-back. With P.pay, the last pass
// (desc) also writes the tile record of each entry's position.
template <typename K, bool SEG>
__global__ void __launch_bounds__(LEGS_SORT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
k_onesweep(const K *__restrict__ kin, const uint32_t *__restrict__ vin, K *__restrict__ kout,
           uint32_t *__restrict__ vout, const uint64_t *__restrict__ count, int64_t capacity, int pass,
           int shift, int rb, const uint32_t *__restrict__ desc, const uint32_t *__restrict__ digit_hist,
           uint64_t *__restrict__ status, uint32_t *__restrict__ counter, CoarsePay P,
           const uint32_t *__restrict__ seg_off)
{
    const bool payload = P.pay != nullptr && desc != nullptr && pass == (int)desc[0] - 1;
    const bool has_vals = vin != nullptr;   // no values: they travel in the key's low bits
    if (desc) {
        shift = (int)desc[2 + 2 * pass];
        rb = (int)desc[3 + 2 * pass];
        if (rb == 0) return;
    }
    constexpr int T = LEGS_SORT_THREADS;
    constexpr int NW = T / LEGS_WAVE;
    constexpr int ITEMS = LEGS_SORT_ITEMS;
    constexpr int PART = LEGS_SORT_PART;
    static_assert(T >= 256 && T % 256 == 0, "one thread per digit");
    __shared__ K s_keys[PART];
    __shared__ uint32_t s_vals[PART];
    __shared__ uint32_t s_wh[NW][256];      // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_lstart[256];      // block-local start of each digit
    __shared__ uint64_t s_gstart[257];      // global position of LDS slot 0 of each digit
    __shared__ uint32_t s_tmp[NW];
    __shared__ int64_t s_part;

    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    const int64_t parts = (m + PART - 1) / PART;
    const uint32_t dmask = (1u << rb) - 1u;    // digit = bits [shift, shift + rb) of the key
    const int tid = threadIdx.x, lane = legs_lane(), wave = tid / LEGS_WAVE;

    // SEG: workgroup b owns partitions [b per, (b + 1) per) in order and keeps
    // the running global start of every digit, seeded from the segment scan
    __shared__ uint64_t s_run[SEG ? 256 : 1];
    int64_t per = 0, iseg = 0;
    if constexpr (SEG) {
        per = (parts + gridDim.x - 1) / gridDim.x;
        if (tid < 256) s_run[tid] = seg_off[(int64_t)blockIdx.x * 256 + tid];
    }
    // look-back: the global start of every digit, an exclusive scan of the
    // pass's digit counts
    __shared__ uint32_t s_dstart[SEG ? 1 : 256];
    if constexpr (!SEG) {
        uint32_t h = 0, incl = 0;
        if (tid < 256) {
            h = digit_hist[pass * 256 + tid];
            incl = wave_incl_add(h);
            if (lane == LEGS_WAVE - 1) s_tmp[wave] = incl;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += s_tmp[w];
            s_dstart[tid] = pre + incl - h;
        }
        __syncthreads();
    }
    for (;;) {
        if constexpr (SEG) {
            if (tid == 0) s_part = iseg < per ? (int64_t)blockIdx.x * per + iseg : parts;
            ++iseg;
        } else {
            if (tid == 0) s_part = (int64_t)atomicAdd(counter, 1u);
        }
        for (int i = tid; i < NW * 256; i += T) (&s_wh[0][0])[i] = 0;
        __syncthreads();
        const int64_t part = s_part;
        if (part >= parts) break;
        const int64_t base = part * PART;
        const int64_t nvalid64 = m - base < PART ? m - base : PART;
        const int nvalid = (int)nvalid64;

        K key[ITEMS];
        uint32_t val[ITEMS];
        uint32_t rank[ITEMS];
        // wave-striped: item i of lane l of wave w is partition element w*64*ITEMS + i*64 + l
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * ITEMS + i * LEGS_WAVE + lane;
            if (e < nvalid) {
                key[i] = kin[base + e];
                val[i] = has_vals ? vin[base + e] : 0u;
            } else {
                key[i] = (K)~(K)0;
                val[i] = 0;
            }
        }
        // rank within the wave: peers with the same digit via 8 ballots
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * ITEMS + i * LEGS_WAVE + lane;
            const bool ok = e < nvalid;
            const uint32_t d = (uint32_t)(key[i] >> shift) & dmask;
            // lanes with the same digit: per bit, the ballot where the bit is set
            // and its complement where it is clear (s: all ones where set)
            const uint64_t okb = legs_ballot(ok);
            uint32_t plo = (uint32_t)okb, phi = (uint32_t)(okb >> 32);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                if (b >= rb) break;
                const int32_t sb = ((int32_t)(d << (31 - b))) >> 31;
                const uint64_t bal = legs_ballot(sb != 0);
                plo &= ~((uint32_t)bal ^ (uint32_t)sb);
                phi &= ~((uint32_t)(bal >> 32) ^ (uint32_t)sb);
            }
            // the lowest peer reserves the run for all of them; an LDS atomic keeps
            // the reservation ordered against the next item's reservation
            const int leader = plo ? __builtin_ctz(plo) : 32 + __builtin_ctz(phi | 0x80000000u);
            uint32_t pre = 0;
            if (ok && lane == leader)
                pre = atomicAdd(&s_wh[wave][d], (uint32_t)(__builtin_popcount(plo) + __builtin_popcount(phi)));
            const uint32_t lbase = (uint32_t)__shfl((int)pre, ok ? leader : lane, LEGS_WAVE);
            rank[i] = lbase + __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
        }
        __syncthreads();
        // per digit (threads 0..255): offsets of each wave, partition total
        // (published at once), block-local digit starts
        uint32_t t = 0, incl = 0, lstart = 0;
        if (tid < 256) {
            const int d = tid;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = s_wh[w][d];
                s_wh[w][d] = t;
                t += c;
            }
            if constexpr (!SEG) st_status(status + part * 256 + d, (part == 0 ? FLAG_INC : FLAG_AGG) | (uint64_t)t);
            incl = t;
#pragma unroll
            for (int off = 1; off < LEGS_WAVE; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
                if (lane >= off) incl += y;
            }
            if (lane == LEGS_WAVE - 1) s_tmp[wave] = incl;
        }
        __syncthreads();
        if (tid < 256) {
            uint32_t wp = 0;
            for (int w = 0; w < wave; ++w) wp += s_tmp[w];
            lstart = wp + incl - t;
            s_lstart[tid] = lstart;
        }
        __syncthreads();
        // scatter into LDS in digit order
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * ITEMS + i * LEGS_WAVE + lane;
            if (e < nvalid) {
                const uint32_t d = (uint32_t)(key[i] >> shift) & dmask;
                const uint32_t pos = s_lstart[d] + s_wh[wave][d] + rank[i];
                s_keys[pos] = key[i];
                if (has_vals) s_vals[pos] = val[i];
            }
        }
        // global start of each digit run: the segment's running start, or a
        // look-back over the partitions before this one
        if (SEG && tid < 256) {
            s_gstart[tid] = s_run[tid] - (uint64_t)lstart;
            s_run[tid] += t;
        } else if (tid < 256) {
            const int d = tid;
            uint64_t excl = 0;
            if (part > 0) {
                // a window of LB predecessors per round trip: their status words
                // are loaded at once, then summed from the nearest outward up to
                // the first inclusive one (or re-read from the first one not yet
                // published)
                constexpr int LB = 4;   // measured: 4 beats 8, 16 and 32 at 1M and 16M keys
                int64_t j = part - 1;
                for (;;) {
                    uint64_t sv[LB];
#pragma unroll
                    for (int q = 0; q < LB; ++q)
                        sv[q] = j - q >= 0 ? ld_status(status + (j - q) * 256 + d) : FLAG_INC;
                    bool done = false;
                    int q = 0;
                    for (; q < LB; ++q) {
                        const uint64_t f = sv[q] & ~VALUE_MASK;
                        if (f == 0) break;               // not published yet: re-read from here
                        excl += sv[q] & VALUE_MASK;
                        if (f == FLAG_INC) { done = true; break; }
                    }
                    if (done) break;
                    j -= q;
                }
                st_status(status + part * 256 + d, FLAG_INC | (excl + t));
            }
            s_gstart[d] = (uint64_t)s_dstart[d] + excl - (uint64_t)lstart;
        }
        __syncthreads();
        // write out digit runs: consecutive lanes, consecutive addresses (positions
        // past the capacity cannot occur when the digit histograms count exactly
        // the stored instances; the test keeps a wrong one in bounds)
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
            const int k = tid + j * T;
            if (k < nvalid) {
                const K kk = s_keys[k];
                const uint32_t d = (uint32_t)(kk >> shift) & dmask;
                const uint64_t gpos = s_gstart[d] + (uint64_t)k;
                if (gpos < (uint64_t)capacity) {
                    if (!payload) kout[gpos] = kk;   // the last coarse pass's keys are not read
                    if (has_vals) vout[gpos] = s_vals[k];
                    // the partition's positions span a narrow window: these gathers stay in cache
                    if (payload) {
                        const uint32_t pv = s_vals[k];
                        P.pay[gpos] = (int64_t)pv < P.G ? P.frecs[pv] : FRec{0u, 0u, 0u, 0u};
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Digit counts of coarse pass `pass` over the partitions of segment
// blockIdx.x (the same segments as the segment passes: per =
// ceil(partitions / gridDim.x)).
__global__ void __launch_bounds__(LEGS_SORT_THREADS)
k_coarse_upsweep(const uint32_t *__restrict__ kin, const uint64_t *__restrict__ count, int64_t capacity,
               const uint32_t *__restrict__ desc, int pass, uint32_t *__restrict__ seg_hist)
{
    constexpr int T = LEGS_SORT_THREADS, PART = LEGS_SORT_PART, ITEMS = LEGS_SORT_ITEMS;
    const int shift = (int)desc[2 + 2 * pass], rb = (int)desc[3 + 2 * pass];
    if (rb == 0) return;
    __shared__ uint32_t s_hist[256];
    const int tid = threadIdx.x;
    if (tid < 256) s_hist[tid] = 0;
    __syncthreads();
    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    const int64_t parts = (m + PART - 1) / PART;
    const int64_t per = (parts + gridDim.x - 1) / gridDim.x;
    const uint32_t dmask = (1u << rb) - 1u;
    for (int64_t i = 0; i < per; ++i) {
        const int64_t part = (int64_t)blockIdx.x * per + i;
        if (part >= parts) break;
        const int64_t base = part * PART;
        const int nvalid = (int)(m - base < PART ? m - base : PART);
        uint32_t k[ITEMS];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
            const int e = tid + q * T;
            k[q] = e < nvalid ? kin[base + e] : 0u;
        }
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) hist_add(s_hist, (k[q] >> shift) & dmask, tid + q * T < nvalid);
    }
    __syncthreads();
    if (tid < 256) seg_hist[(int64_t)blockIdx.x * 256 + tid] = s_hist[tid];
}

// Start of every digit run of every segment: the digit's global start plus the
// counts of the segments before. One workgroup per digit, one thread per
// segment (nseg <= LEGS_SEG_MAX).
__global__ void __launch_bounds__(LEGS_SEG_MAX)
k_seg_scan(const uint32_t *__restrict__ seg_hist, int nseg, const uint32_t *__restrict__ hist,
           const uint32_t *__restrict__ desc, int pass, uint32_t *__restrict__ seg_off)
{
    if (desc[3 + 2 * pass] == 0) return;
    __shared__ uint32_t s_w[LEGS_SEG_MAX / LEGS_WAVE];
    __shared__ uint32_t s_d[256 / LEGS_WAVE];
    const int d = blockIdx.x, sg = threadIdx.x;
    const int lane = legs_lane(), wave = sg / LEGS_WAVE;
    if (sg < 256) {   // the digit's global start: the pass's counts of the digits below it
        uint32_t h = sg < d ? hist[pass * 256 + sg] : 0u;
#pragma unroll
        for (int off = LEGS_WAVE / 2; off > 0; off >>= 1) h += __shfl_xor(h, off, LEGS_WAVE);
        if (lane == 0) s_d[wave] = h;
    }
    const uint32_t x = sg < nseg ? seg_hist[(int64_t)sg * 256 + d] : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int w = 0; w < 256 / LEGS_WAVE; ++w) pre += s_d[w];
    for (int w = 0; w < wave; ++w) pre += s_w[w];
    if (sg < nseg) seg_off[(int64_t)sg * 256 + d] = pre + incl - x;
}

// ---- depth order of the G-views ---------------------------------------------------

// key = (view << 32) | bits(depth) for visible G-views (culled ones sort last,
// they emit nothing); value = G-view index. With vbits > 0 the value travels
// in the key's low bits, (key << vbits) | index (culled: all ones), and the
// digits of the passes start at bit vbits. Also stores G for the sort and
// counts the digit histograms of its npass passes into hist (cleared before):
// each workgroup takes chunks of ORDER_RUN rows of ORDER_THREADS G-views,
// loads a chunk's inputs at once, counts in LDS (hist_add for the clustered
// digits) and flushes its counts once.
constexpr int ORDER_THREADS = 1024, ORDER_RUN = 4;   // measured: 4 waves per SIMD beat 1 (256 x 16)

__global__ void __launch_bounds__(ORDER_THREADS)
k_order_keys(const uint32_t *__restrict__ ntiles, const float *__restrict__ depth, int64_t n,
             int64_t G, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
             uint64_t *__restrict__ gcount, int npass, uint32_t *__restrict__ hist, int vbits)
{
    constexpr int NT = ORDER_THREADS, RUN = ORDER_RUN;
    __shared__ uint32_t s_h[LEGS_SORT_MAX_PASSES][256];
    for (int i = threadIdx.x; i < LEGS_SORT_MAX_PASSES * 256; i += NT) (&s_h[0][0])[i] = 0;
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) *gcount = (uint64_t)G;
    const bool narrow = G <= (int64_t)0xffffffffll;
    const int64_t chunk = (int64_t)NT * RUN;
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < G; base += (int64_t)gridDim.x * chunk) {
        uint32_t nt[RUN];
        float dp[RUN];
#pragma unroll
        for (int i = 0; i < RUN; ++i) {
            const int64_t gv = base + NT * i + threadIdx.x;
            nt[i] = gv < G ? ntiles[gv] : 0u;
            dp[i] = gv < G ? depth[gv] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < RUN; ++i) {
            const int64_t gv = base + NT * i + threadIdx.x;
            const bool ok = gv < G;
            uint64_t key = ~0ull;
            if (ok) {
                const uint64_t v = narrow ? (uint64_t)((uint32_t)gv / (uint32_t)n) : (uint64_t)(gv / n);
                if (nt[i]) key = (v << 32) | __float_as_uint(dp[i]);
                if (vbits > 0) {
                    if (nt[i]) key = (key << vbits) | (uint64_t)gv;
                } else {
                    vals[gv] = (uint32_t)gv;
                }
                keys[gv] = key;
            }
            for (int p = 0; p < npass; ++p) {
                // the low two bytes of a depth are spread, the higher ones cluster
                const uint32_t d = (uint32_t)(key >> (vbits + 8 * p)) & 255u;
                if (p >= 2) hist_add(s_h[p], d, ok);
                else if (ok) atomicAdd(&s_h[p][d], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += NT) {
        const uint32_t c = (&s_h[0][0])[i];
        if (c) atomicAdd(&hist[i], c);
    }
}

// Super-tile edge in tiles: 8 x 4 tiles, one bit each of a 32-bit mask.
constexpr int SX = 8, SY = 4, SUPER_TILES = SX * SY;
static_assert(SUPER_TILES == 32, "one mask bit per tile of a super-tile");
// Entries of the coarse lists per unit of the compaction (one wave each).
constexpr int UNIT = LEGS_COMPACT_UNIT;

// Tile and super-tile records and the per-view position ranges of the
// depth-ordered G-views, and the tile and super-tile instance counts of each
// block of LEGS_PROJ_BLOCK positions.
__global__ void __launch_bounds__(LEGS_PROJ_BLOCK)
k_sorted_records(const uint32_t *__restrict__ perm, const uint64_t *__restrict__ okeys, int vbits,
                 const int4 *__restrict__ box, int64_t n, int64_t G, const legs_view *__restrict__ sviews, int tile,
                 FRec *__restrict__ frecs, GRec *__restrict__ crecs, uint64_t *__restrict__ vrange,
                 uint64_t *__restrict__ block_counts, uint64_t *__restrict__ cblock_counts)
{
    const int64_t pos = (int64_t)blockIdx.x * LEGS_PROJ_BLOCK + threadIdx.x;
    uint64_t c = 0, cc = 0;
    if (pos < G) {
        // culled G-views (no tiles) carry the all-ones key and sort last; the key of a
        // visible one holds its depth bits, and its tile count follows from its box,
        // so the box is the only gather
        const uint64_t packed = okeys[pos];
        const uint64_t key = packed >> vbits;      // (view << 32) | depth bits
        FRec f = {0u, 0u, 0u, 0u};
        GRec r = {(uint32_t)pos, 0u, 0u, 0u};
        if (packed != ~0ull) {
            const int64_t gv = vbits > 0 ? (int64_t)(packed & ((1ull << vbits) - 1)) : (int64_t)perm[pos];
            const int64_t v = gv / n;
            const int4 bx = box[gv];
            const legs_view &sw = sviews[v];
            const int tx0 = bx.x / tile, tx1 = bx.y / tile, ty0 = bx.z / tile, ty1 = bx.w / tile;
            c = (uint64_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
            f.gid = (uint32_t)(gv - v * n);
            f.dbits = (uint32_t)key;
            f.xy = (uint32_t)tx0 | ((uint32_t)ty0 << 16);
            f.wh = (uint32_t)(tx1 - tx0 + 1) | ((uint32_t)(ty1 - ty0 + 1) << 16);
            const int sx0 = tx0 / SX, sx1 = tx1 / SX, sy0 = ty0 / SY, sy1 = ty1 / SY;
            r.cnt = (uint32_t)((sx1 - sx0 + 1) * (sy1 - sy0 + 1));
            r.base = (uint32_t)(sw.tile_offset + (int64_t)sy0 * sw.tiles_x + sx0);
            r.rwtx = (uint32_t)(sx1 - sx0 + 1) | ((uint32_t)sw.tiles_x << 16);
            cc = r.cnt;
            // first and last position of each view (visible G-views sort by view)
            const uint64_t kv = key >> 32;
            if (pos == 0 || ((okeys[pos - 1] >> vbits) >> 32) != kv) vrange[2 * kv] = (uint64_t)pos;
            if (pos == G - 1 || ((okeys[pos + 1] >> vbits) >> 32) != kv) vrange[2 * kv + 1] = (uint64_t)pos + 1;
        }
        frecs[pos] = f;
        crecs[pos] = r;
    }
#pragma unroll
    for (int off = LEGS_WAVE / 2; off > 0; off >>= 1) {
        c += __shfl_down(c, off, LEGS_WAVE);
        cc += __shfl_down(cc, off, LEGS_WAVE);
    }
    __shared__ uint64_t s_w[2][LEGS_PROJ_BLOCK / LEGS_WAVE];
    if (legs_lane() == 0) {
        s_w[0][threadIdx.x / LEGS_WAVE] = c;
        s_w[1][threadIdx.x / LEGS_WAVE] = cc;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint64_t t = 0;
        for (int w = 0; w < LEGS_PROJ_BLOCK / LEGS_WAVE; ++w) t += s_w[threadIdx.x][w];
        (threadIdx.x == 0 ? block_counts : cblock_counts)[blockIdx.x] = t;
    }
}

// The coarse stream written out: each G-view's super-tile rectangle,
// row-major, at its offset in the stream (the first ccap entries kept), key =
// super-tile id, value = position. The block's entries are spread evenly over
// its threads (consecutive threads, consecutive entries); each finds its
// G-view by binary search over the block's scan in LDS.
__global__ void __launch_bounds__(LEGS_PROJ_BLOCK)
k_coarse_emit(const GRec *__restrict__ crecs, const uint64_t *__restrict__ coff, int64_t G, int64_t ccap,
              uint32_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    static_assert(LEGS_PROJ_BLOCK == 256, "offsets per block of 256 positions");
    __shared__ uint64_t s_start[257];
    __shared__ uint64_t s_w[4];
    __shared__ uint32_t s_base[256], s_rwtx[256];
    const int64_t pos0 = (int64_t)blockIdx.x * 256;
    const GRec r = pos0 + threadIdx.x < G ? crecs[pos0 + threadIdx.x] : GRec{0u, 0u, 0u, 0u};
    s_base[threadIdx.x] = r.base;
    s_rwtx[threadIdx.x] = r.rwtx;
    block_scan_256<256>(r.cnt, s_start, s_w);
    const uint64_t o0 = coff[blockIdx.x];
    const uint64_t tot = s_start[256];
    const uint64_t lim = (uint64_t)ccap > o0 ? (uint64_t)ccap - o0 : 0u;
    const uint32_t n = (uint32_t)(tot < lim ? tot : lim);
    for (uint32_t e = threadIdx.x; e < n; e += 256) {
        int lo = 0, hi = 255;   // the last G-view starting at or before e (it has entries)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_start[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const uint32_t k = e - (uint32_t)s_start[lo];
        const uint32_t rw = s_rwtx[lo] & 0xffffu, stx = s_rwtx[lo] >> 16;
        const uint32_t y = k / rw, x = k - y * rw;
        keys[o0 + e] = s_base[lo] + y * stx + x;
        vals[o0 + e] = (uint32_t)(pos0 + lo);
    }
}

// ---- per-tile counts of the depth-ordered streams ------------------------------

// Two streams are counted per cell of a 2D difference array: the tile stream
// (each G-view's tile rectangle, the first `capacity` instances kept) on the
// tile grids of the views, and the coarse stream (each G-view's super-tile
// rectangle, the first `ccap` kept) on the super-tile grids: +1 / -1 at the
// corners of each rectangle, then prefix sums along the rows and the columns.
// A G-view cut by its capacity contributes its first cells in row-major order
// (full rows plus one partial row). The counts give the list ranges (and the
// digit histograms of the coarse passes) without reading any instance. Every
// kernel below handles both grids at once (grid 0: tiles, grid 1: super-tiles).
// +1 / -1 at the corners of a rectangle (view-local cell coordinates).
__device__ __forceinline__ void diff_rect(uint32_t *g, int W, int H, int x0, int x1, int y0, int y1)
{
    atomicAdd(g + y0 * W + x0, 1u);
    if (x1 + 1 < W) atomicAdd(g + y0 * W + x1 + 1, 0xffffffffu);
    if (y1 + 1 < H) atomicAdd(g + (y1 + 1) * W + x0, 0xffffffffu);
    if (x1 + 1 < W && y1 + 1 < H) atomicAdd(g + (y1 + 1) * W + x1 + 1, 1u);
}

// Adds a rectangle cut to its first `keep` cells.
__device__ __forceinline__ void diff_rect_kept(uint32_t *g, int W, int H, int x0, int y0, int w, int h,
                                               uint64_t keep)
{
    if (keep >= (uint64_t)w * (uint64_t)h) {
        diff_rect(g, W, H, x0, x0 + w - 1, y0, y0 + h - 1);
    } else {
        const int full = (int)(keep / (uint64_t)w), rem = (int)(keep % (uint64_t)w);
        if (full > 0) diff_rect(g, W, H, x0, x0 + w - 1, y0, y0 + full - 1);
        if (rem > 0) diff_rect(g, W, H, x0, x0 + rem - 1, y0 + full, y0 + full);
    }
}

constexpr int TILE_LDS_CELLS = 16384;   // tile grids with at most this many cells count in LDS
constexpr int SUPER_LDS_CELLS = 4096;   // super-tile grids likewise

// One of the two count grids.
struct CountGrid {
    const legs_view *views;   // the tile or super-tile views
    uint32_t *count;          // [T] cells (at most T of them)
    uint32_t *partial;        // [LEGS_TILE_CHUNKS][T] per-workgroup LDS grids
    uint32_t *ranges;         // [T][2]
    const uint32_t *desc;     // digit layout of passes over these cells (NULL: none)
    uint32_t *hist;           // digit histograms of those passes
};

// Workgroup (c, v) adds the rectangles of view v's G-views in position blocks
// c, c + gridDim.x, ... to LDS copies of the view's tile and super-tile grids
// and stores them in the partial grids of chunk c (grids with more cells than
// fit add straight into the count arrays with atomics); k_count_merge then sums
// the partial grids. Hot corner cells cost LDS atomics instead of global ones.
// The G-view whose tile instances reach past the capacity stores its position
// and how many of its tiles fit in cut (at most one G-view does).
__global__ void __launch_bounds__(256)
k_count_corners(const FRec *__restrict__ frecs, const GRec *__restrict__ crecs,
                const uint64_t *__restrict__ goff, const uint64_t *__restrict__ coff,
                const uint64_t *__restrict__ vrange, int64_t G, int64_t capacity, int64_t ccap, int64_t T,
                const uint64_t *__restrict__ count, const uint64_t *__restrict__ ccount,
                CountGrid g0, CountGrid g1, uint64_t *__restrict__ cut)
{
    // offsets inside the streams only matter when a stream overflows its capacity
    const bool scan = *count > (uint64_t)capacity || *ccount > (uint64_t)ccap;
    __shared__ uint32_t s_grid[TILE_LDS_CELLS];
    __shared__ uint32_t s_sgrid[SUPER_LDS_CELLS];
    __shared__ uint64_t s_start[257], s_cstart[257];
    __shared__ uint64_t s_w[4];
    const int v = blockIdx.y;
    const legs_view vw = g0.views[v], sw = g1.views[v];
    const int W = vw.tiles_x, H = vw.tiles_y, SWd = sw.tiles_x, SH = sw.tiles_y;
    const int ncell = W * H, nscell = SWd * SH;
    const bool lds = ncell <= TILE_LDS_CELLS, slds = nscell <= SUPER_LDS_CELLS;
    uint32_t *g = lds ? s_grid : g0.count + vw.tile_offset;
    uint32_t *sg = slds ? s_sgrid : g1.count + sw.tile_offset;
    if (lds)
        for (int i = threadIdx.x; i < ncell; i += 256) s_grid[i] = 0u;
    if (slds)
        for (int i = threadIdx.x; i < nscell; i += 256) s_sgrid[i] = 0u;
    const int64_t p0 = (int64_t)vrange[2 * v], p1 = (int64_t)vrange[2 * v + 1];
    __syncthreads();
    if (p1 > p0) {
        for (int64_t b = p0 / 256 + blockIdx.x; b <= (p1 - 1) / 256; b += gridDim.x) {
            const int64_t pos = b * 256 + threadIdx.x;
            // the whole block is scanned: its offsets count the positions of other views too
            const FRec f = pos < G ? frecs[pos] : FRec{0u, 0u, 0u, 0u};
            const GRec r = pos < G ? crecs[pos] : GRec{0u, 0u, 0u, 0u};
            const uint32_t fw = f.wh & 0xffffu, fh = f.wh >> 16;
            if (scan) {
                block_scan_256<256>((uint64_t)fw * fh, s_start, s_w);
                block_scan_256<256>(r.cnt, s_cstart, s_w);
            }
            if (pos >= p0 && pos < p1 && fw) {
                const uint32_t cnt = fw * fh;
                const uint64_t off = scan ? goff[b] + s_start[threadIdx.x] : 0u;
                if (off <= (uint64_t)capacity && off + cnt > (uint64_t)capacity) {
                    cut[0] = (uint64_t)pos;
                    cut[1] = (uint64_t)capacity - off;
                }
                if (off < (uint64_t)capacity)
                    diff_rect_kept(g, W, H, (int)(f.xy & 0xffffu), (int)(f.xy >> 16), (int)fw, (int)fh,
                                   (uint64_t)capacity - off);
                const uint64_t co = scan ? coff[b] + s_cstart[threadIdx.x] : 0u;
                if (co < (uint64_t)ccap) {
                    const int local = (int)((int64_t)r.base - sw.tile_offset);
                    const int cw = (int)(r.rwtx & 0xffffu);
                    diff_rect_kept(sg, SWd, SH, local % SWd, local / SWd, cw, (int)(r.cnt / (uint32_t)cw),
                                   (uint64_t)ccap - co);
                }
            }
            if (scan) __syncthreads();   // s_start is rewritten by the next block's scan
        }
    }
    __syncthreads();
    if (lds) {
        uint32_t *out = g0.partial + (int64_t)blockIdx.x * T + vw.tile_offset;
        for (int i = threadIdx.x; i < ncell; i += 256) out[i] = s_grid[i];
    }
    if (slds) {
        uint32_t *out = g1.partial + (int64_t)blockIdx.x * T + sw.tile_offset;
        for (int i = threadIdx.x; i < nscell; i += 256) out[i] = s_sgrid[i];
    }
}

// Adds the partial grids of the grids counted in LDS to the (cleared) counts:
// chunk group blockIdx.y sums chunks blockIdx.y, blockIdx.y + gridDim.y, ...
// of each cell. T may exceed a grid's cells (the super-tile grids): cells
// past its last view are left alone.
__global__ void __launch_bounds__(256)
k_count_merge(int nch, int64_t T, int n_views, CountGrid g0, CountGrid g1)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < 2 * T; i += (int64_t)gridDim.x * 256) {
        const bool sup = i >= T;
        const int64_t t = sup ? i - T : i;
        const CountGrid &cg = sup ? g1 : g0;
        const legs_view &vw = cg.views[legs_view_of_tile(cg.views, n_views, t)];
        const int64_t ncell = (int64_t)vw.tiles_x * vw.tiles_y;
        if (ncell > (sup ? SUPER_LDS_CELLS : TILE_LDS_CELLS) || t - vw.tile_offset >= ncell) continue;
        uint32_t acc = 0;
#pragma unroll 8
        for (int c = blockIdx.y; c < nch; c += gridDim.y) acc += cg.partial[(int64_t)c * T + t];
        if (acc) atomicAdd(cg.count + t, acc);
    }
}

// Row, then column inclusive prefix sums of the difference grid of view
// blockIdx.x in grid blockIdx.y (one workgroup per view and grid, a wave per
// row or column), which turns the corner counts into per-cell counts.
__global__ void __launch_bounds__(1024)
k_count_prefix(CountGrid g0, CountGrid g1)
{
    const CountGrid &cg = blockIdx.y ? g1 : g0;
    const legs_view vw = cg.views[blockIdx.x];
    const int lane = legs_lane(), wave = (int)(threadIdx.x / LEGS_WAVE);
    constexpr int NW = 1024 / LEGS_WAVE;
    uint32_t *base = cg.count + vw.tile_offset;
    for (int y = wave; y < vw.tiles_y; y += NW) {
        uint32_t *r = base + (int64_t)y * vw.tiles_x;
        uint32_t carry = 0;
        for (int x0 = 0; x0 < vw.tiles_x; x0 += LEGS_WAVE) {
            const int x = x0 + lane;
            uint32_t incl = wave_incl_add(x < vw.tiles_x ? r[x] : 0u);
            if (x < vw.tiles_x) r[x] = carry + incl;
            carry += (uint32_t)__shfl((int)incl, LEGS_WAVE - 1, LEGS_WAVE);
        }
    }
    __syncthreads();   // the rows are done (and visible to the workgroup)
    for (int x = wave; x < vw.tiles_x; x += NW) {
        uint32_t *col = base + x;
        uint32_t carry = 0;
        for (int y0 = 0; y0 < vw.tiles_y; y0 += LEGS_WAVE) {
            const int y = y0 + lane;
            uint32_t incl = wave_incl_add(y < vw.tiles_y ? col[(int64_t)y * vw.tiles_x] : 0u);
            if (y < vw.tiles_y) col[(int64_t)y * vw.tiles_x] = carry + incl;
            carry += (uint32_t)__shfl((int)incl, LEGS_WAVE - 1, LEGS_WAVE);
        }
    }
}

// Cell at position t of the list order: the cell itself, except for the
// super-tile grid when its coarse passes take the top bits first and the low
// byte last (desc[1] = S, the number of super-tiles): its lists are then
// ordered by (low byte, id >> 8), and position t holds super-tile
// 256 h + l with l, h from t (low bytes below S mod 256 hold one more id).
__device__ __forceinline__ int64_t list_cell(int64_t t, const uint32_t *__restrict__ desc)
{
    const int64_t S = desc ? (int64_t)desc[1] : 0;
    if (S <= 256 || t >= S) return t;
    const int64_t hf = S >> 8, r = S & 255;
    int64_t l, h;
    if (t < r * (hf + 1)) {
        l = t / (hf + 1);
        h = t - l * (hf + 1);
    } else {
        const int64_t u = t - r * (hf + 1);
        l = r + u / hf;
        h = u - (l - r) * hf;
    }
    return (h << 8) | l;
}

// List ranges [start, start + count) of every cell, one workgroup per grid:
// grid 0's cells in order, grid 1's in list order (list_cell) with the digit
// histograms of the coarse passes; a third workgroup numbers the units of the
// super-tile lists, ceil(count / UNIT) per super-tile in id order (uoff[T] =
// their number).
__global__ void __launch_bounds__(1024)
k_count_lists(int64_t T, CountGrid g0, CountGrid g1, uint32_t *__restrict__ uoff)
{
    if (blockIdx.x == 2) {
        const uint32_t t = scan_rounds<uint32_t>(
            T, [&](int64_t c) { return (g1.count[c] + UNIT - 1) / UNIT; },
            [&](int64_t c, uint32_t e, uint32_t) { uoff[c] = e; });
        if (threadIdx.x == 0) uoff[T] = t;
        return;
    }
    const CountGrid &cg = blockIdx.x ? g1 : g0;
    __shared__ uint32_t s_h[LEGS_SORT_MAX_PASSES][256];
    const int npass = cg.desc ? (int)cg.desc[0] : 0;
    for (int i = threadIdx.x; i < LEGS_SORT_MAX_PASSES * 256; i += 1024) (&s_h[0][0])[i] = 0;
    __syncthreads();
    scan_rounds<uint32_t>(
        T, [&](int64_t t) { return cg.count[list_cell(t, cg.desc)]; },
        [&](int64_t t, uint32_t e, uint32_t x) {
            const int64_t c = list_cell(t, cg.desc);
            cg.ranges[2 * c] = e;
            cg.ranges[2 * c + 1] = e + x;
            if (x)
                for (int p = 0; p < npass; ++p)
                    atomicAdd(&s_h[p][(uint32_t)(c >> cg.desc[2 + 2 * p]) & ((1u << cg.desc[3 + 2 * p]) - 1u)], x);
        });
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += 1024) {
        const uint32_t c = (&s_h[0][0])[i];
        if (c) atomicAdd(&cg.hist[i], c);
    }
}

// ---- two-level binning: super-tile lists, compacted into tile lists ---------

// Super-tile grids of the views (SX x SY tiles each, numbered after one
// another like the tile grids) and the digit layout of the coarse passes:
// ceil(bits / 8) passes over the bits of the super-tile id: one pass over the
// whole id; two passes over the top bits, then the low byte (lists ordered
// by (low byte, id >> 8), see list_cell); more, even digits from the lowest.
// The other threads clear the digit histograms and pass counters, the
// capacity cut (no G-view cut) and the per-view position ranges, and every
// workgroup clears its share of the nclear cell counts at clear.
struct SuperViewArgs {
    const legs_view *views;
    int n_views;
    legs_view *sv;
    uint32_t *desc, *hist, *counters;
    uint64_t *cut, *vrange;
    uint32_t *clear;
    int64_t nclear;
};

// The share of workgroup `block` of `blocks`.
__device__ __forceinline__ void super_views_part(const SuperViewArgs &a, int64_t block, int64_t blocks)
{
    for (int64_t i = block * 256 + threadIdx.x; i < a.nclear; i += blocks * 256) a.clear[i] = 0u;
    if (block != 0) return;
    for (int i = threadIdx.x; i < LEGS_SORT_MAX_PASSES * 256; i += 256) a.hist[i] = 0u;
    for (int i = threadIdx.x; i < 2 * a.n_views; i += 256) a.vrange[i] = 0u;
    if (threadIdx.x < 16) a.counters[threadIdx.x] = 0u;
    if (threadIdx.x < 2) a.cut[threadIdx.x] = ~0ull;
    if (threadIdx.x != 0) return;
    const int n_views = a.n_views;
    const legs_view *views = a.views;
    legs_view *sv = a.sv;
    uint32_t *desc = a.desc;
    int64_t off = 0;
    for (int v = 0; v < n_views; ++v) {
        legs_view w = views[v];
        w.tiles_x = (w.tiles_x + SX - 1) / SX;
        w.tiles_y = (w.tiles_y + SY - 1) / SY;
        w.tile_offset = off;
        off += (int64_t)w.tiles_x * w.tiles_y;
        sv[v] = w;
    }
    int bits = 1;
    while (bits < 32 && (1ll << bits) < off) ++bits;
    const int np = (bits + 7) / 8;
    desc[0] = (uint32_t)np;
    desc[1] = np == 2 ? (uint32_t)off : 0u;
    for (int p = 0, sh = 0; p < LEGS_SORT_MAX_PASSES; ++p) {
        const int w = p < np ? bits / np + (p < bits % np ? 1 : 0) : 0;
        desc[2 + 2 * p] = (uint32_t)sh;
        desc[3 + 2 * p] = (uint32_t)w;
        sh += w;
    }
    if (np == 2) {
        // top bits first, low byte last: the last pass then reads runs of 256
        // consecutive super-tiles (one or two views), whose entries' positions
        // are dense, so its record gathers stay local
        desc[2] = 8u;
        desc[3] = (uint32_t)(bits - 8);
        desc[4] = 0u;
        desc[5] = 8u;
    }
}

// The set-up of the depth-first binning in one launch: the G-view sort's
// scratch cleared (sort_clear_part) and the super-tile views with the
// clears of the counting and coarse scratch (super_views_part, whose
// single-workgroup part goes to the last workgroup).
__global__ void __launch_bounds__(256) k_bin_setup(SortClearArgs a, SuperViewArgs b)
{
    sort_clear_part(a, blockIdx.x, gridDim.x);
    super_views_part(b, gridDim.x - 1 - blockIdx.x, gridDim.x);
}

// What a wave needs of its unit: the list entries [e0, e1), the super-tile's
// first tile (view-local) and the view's tile grid.
struct UnitCtx {
    uint32_t e0, e1;
    int tx0, ty0, tiles_x, tiles_y;
    int64_t toff;
};

__device__ __forceinline__ UnitCtx unit_ctx(uint32_t u, const uint32_t *__restrict__ uoff, int64_t n,
                                            const uint32_t *__restrict__ cranges,
                                            const legs_view *__restrict__ sviews,
                                            const legs_view *__restrict__ views, int n_views)
{
    int64_t lo = 0, hi = n - 1;   // the last super-tile whose first unit is <= u
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (uoff[mid] <= u) lo = mid; else hi = mid - 1;
    }
    const int64_t st = lo;
    const int v = legs_view_of_tile(sviews, n_views, st);
    const int stx = sviews[v].tiles_x;
    const int local = (int)(st - sviews[v].tile_offset);
    UnitCtx c;
    c.ty0 = (local / stx) * SY;
    c.tx0 = (local - (local / stx) * stx) * SX;
    c.e0 = cranges[2 * st] + (u - uoff[st]) * UNIT;
    const uint32_t end = cranges[2 * st + 1];
    c.e1 = c.e0 + UNIT < end ? c.e0 + UNIT : end;
    c.tiles_x = views[v].tiles_x;
    c.tiles_y = views[v].tiles_y;
    c.toff = views[v].tile_offset;
    return c;
}

// Descriptor of every unit (its super-tile found by binary search over the
// unit offsets), so that each compaction wave starts from one load.
__global__ void __launch_bounds__(256)
k_unit_desc(const uint32_t *__restrict__ uoff, int64_t n, const uint32_t *__restrict__ cranges,
            const legs_view *__restrict__ sviews, const legs_view *__restrict__ views, int n_views,
            UnitCtx *__restrict__ udesc)
{
    const uint32_t nunits = uoff[n];
    for (uint32_t u = blockIdx.x * 256 + threadIdx.x; u < nunits; u += gridDim.x * 256)
        udesc[u] = unit_ctx(u, uoff, n, cranges, sviews, views, n_views);
}

// Tiles of the super-tile at (tx0, ty0) that the record's rectangle covers:
// bit (ty - ty0) * SX + (tx - tx0). The G-view at position cut[0] keeps only
// its first cut[1] tiles in row-major order, the ones after it none (their
// instances lie past the capacity).
__device__ __forceinline__ uint32_t entry_mask(uint32_t pos, const FRec &r, const UnitCtx &c, uint64_t cpos,
                                               uint64_t ckeep)
{
    if ((uint64_t)pos > cpos) return 0u;
    const int x0 = (int)(r.xy & 0xffffu), y0 = (int)(r.xy >> 16);
    const int w = (int)(r.wh & 0xffffu), h = (int)(r.wh >> 16);
    const int cx0 = max(x0 - c.tx0, 0), cx1 = min(x0 + w - 1 - c.tx0, SX - 1);
    const int cy0 = max(y0 - c.ty0, 0), cy1 = min(y0 + h - 1 - c.ty0, SY - 1);
    if (w == 0 || cx0 > cx1 || cy0 > cy1) return 0u;
    const uint32_t cols = (0xffu << cx0) & (0xffu >> (SX - 1 - cx1));
    const uint32_t rows = (0x01010101u << (SX * cy0)) & (0x01010101u >> (SX * (SY - 1 - cy1)));
    uint32_t m = cols * rows;
    if ((uint64_t)pos == cpos) {
        const int kr = (int)(ckeep / (uint64_t)w), kc = (int)(ckeep % (uint64_t)w);
        for (int y = 0; y < SY; ++y) {
            const int r_ = c.ty0 + y - y0;   // row of the rectangle
            uint32_t keep_cols;
            if (r_ < kr) {
                keep_cols = 0xffu;
            } else if (r_ > kr) {
                keep_cols = 0u;
            } else {
                const int lim = x0 + kc - c.tx0;   // columns cx < lim are kept
                keep_cols = lim <= 0 ? 0u : (lim >= SX ? 0xffu : (0xffu >> (SX - lim)));
            }
            m &= ~((~keep_cols & 0xffu) << (SX * y));
        }
    }
    return m;
}

// Counts of each of the 32 tiles in each unit: ucnt[u * 32 + b].
__global__ void __launch_bounds__(256)
k_compact_count(const uint32_t *__restrict__ clist0, const uint32_t *__restrict__ clist1,
                const uint32_t *__restrict__ desc, const uint32_t *__restrict__ uoff, int64_t n,
                const UnitCtx *__restrict__ udesc, const FRec *__restrict__ pay, int64_t G,
                const uint64_t *__restrict__ cut, uint32_t *__restrict__ ucnt)
{
    // pass p of the coarse sort writes buffer p % 2
    const uint32_t *clist = ((desc[0] - 1u) & 1u) ? clist1 : clist0;
    const int lane = legs_lane();
    const uint32_t nunits = uoff[n];
    const uint64_t cpos = cut[0], ckeep = cut[1];
    const uint32_t nw = gridDim.x * (256 / LEGS_WAVE);
    for (uint32_t u = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * (256 / LEGS_WAVE) + threadIdx.x / LEGS_WAVE));
         u < nunits; u += nw) {
        const UnitCtx c = udesc[u];
        uint32_t cnt[SUPER_TILES];
#pragma unroll
        for (int b = 0; b < SUPER_TILES; ++b) cnt[b] = 0;
        for (uint32_t e0 = c.e0; e0 < c.e1; e0 += LEGS_WAVE) {
            const uint32_t e = e0 + lane;
            uint32_t m = 0;
            if (e < c.e1) {
                const uint32_t pos = clist[e];
                if ((int64_t)pos < G) m = entry_mask(pos, pay[e], c, cpos, ckeep);
            }
#pragma unroll
            for (int b = 0; b < SUPER_TILES; ++b) cnt[b] += (uint32_t)__popcll(legs_ballot((m >> b) & 1u));
        }
        uint32_t mine = 0;
#pragma unroll
        for (int b = 0; b < SUPER_TILES; ++b) mine = lane == b ? cnt[b] : mine;
        if (lane < SUPER_TILES) ucnt[(int64_t)u * SUPER_TILES + lane] = mine;
    }
}

// Per super-tile (one wave each): the unit counts of each of its tiles become
// exclusive offsets, starting from the tile's range start.
__global__ void __launch_bounds__(256)
k_compact_scan(const uint32_t *__restrict__ uoff, int64_t n, const legs_view *__restrict__ sviews,
               const legs_view *__restrict__ views, int n_views, const uint32_t *__restrict__ ranges,
               uint32_t *__restrict__ ucnt)
{
    const int lane = legs_lane();
    const uint32_t nunits = uoff[n];
    const int64_t nw = (int64_t)gridDim.x * (256 / LEGS_WAVE);
    for (int64_t st = (int64_t)blockIdx.x * (256 / LEGS_WAVE) + threadIdx.x / LEGS_WAVE; st < n; st += nw) {
        const uint32_t u0 = uoff[st], u1 = uoff[st + 1];
        if (u0 >= nunits) break;   // no units from here on
        if (u0 >= u1) continue;
        const int v = legs_view_of_tile(sviews, n_views, st);
        const int stx = sviews[v].tiles_x;
        const int local = (int)(st - sviews[v].tile_offset);
        const int ty0 = (local / stx) * SY, tx0 = (local - (local / stx) * stx) * SX;
        const legs_view &vw = views[v];
        uint32_t start = 0;
        if (lane < SUPER_TILES) {
            const int tx = tx0 + lane % SX, ty = ty0 + lane / SX;
            if (tx < vw.tiles_x && ty < vw.tiles_y)
                start = ranges[2 * (vw.tile_offset + (int64_t)ty * vw.tiles_x + tx)];
        }
        uint32_t carry[SUPER_TILES];
#pragma unroll
        for (int b = 0; b < SUPER_TILES; ++b) carry[b] = (uint32_t)__builtin_amdgcn_readlane((int)start, b);
        for (uint32_t ub = u0; ub < u1; ub += LEGS_WAVE) {
            const uint32_t u = ub + lane;
            const bool ok = u < u1;
            uint4 q[SUPER_TILES / 4];
            uint4 *row = reinterpret_cast<uint4 *>(ucnt + (int64_t)u * SUPER_TILES);
#pragma unroll
            for (int k = 0; k < SUPER_TILES / 4; ++k) q[k] = ok ? row[k] : make_uint4(0u, 0u, 0u, 0u);
            uint32_t *x = reinterpret_cast<uint32_t *>(q);
#pragma unroll
            for (int b = 0; b < SUPER_TILES; ++b) {
                const uint32_t incl = wave_incl_add(x[b]);
                const uint32_t excl = carry[b] + incl - x[b];
                carry[b] += (uint32_t)__builtin_amdgcn_readlane((int)incl, LEGS_WAVE - 1);
                x[b] = excl;
            }
            if (ok)
#pragma unroll
                for (int k = 0; k < SUPER_TILES / 4; ++k) row[k] = q[k];
        }
    }
}

// Writes the tile lists: each wave takes a unit and holds its entries' tile
// masks, one entry per lane and round of 64. Per tile, the entries covering
// it get their rank among the unit's hits (ballot per round); their (id,
// depth) pairs are placed in rank order in an LDS row of the wave, which is
// then stored as one contiguous run of the tile's list with all lanes (ids,
// and the keys unless keys is NULL). Four tiles are staged per LDS round trip.
__global__ void __launch_bounds__(256)
k_compact_write(const uint32_t *__restrict__ clist0, const uint32_t *__restrict__ clist1,
                const uint32_t *__restrict__ desc, const uint32_t *__restrict__ uoff, int64_t n,
                const UnitCtx *__restrict__ udesc, const FRec *__restrict__ pay, int64_t G,
                const uint64_t *__restrict__ cut, const uint32_t *__restrict__ ucnt, int64_t capacity,
                uint64_t *__restrict__ keys, uint32_t *__restrict__ ids)
{
    constexpr int NQ = UNIT / LEGS_WAVE;
    constexpr int TB = 4;                                   // tiles per LDS round trip
    __shared__ uint2 s_run[256 / LEGS_WAVE][TB][UNIT];      // (id, depth bits) of the hits, in order
    const uint32_t *clist = ((desc[0] - 1u) & 1u) ? clist1 : clist0;
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    uint2(*run)[UNIT] = s_run[wave];
    const uint32_t nunits = uoff[n];
    const uint64_t cpos = cut[0], ckeep = cut[1];
    const uint32_t nw = gridDim.x * (256 / LEGS_WAVE);
    for (uint32_t u = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x * (256 / LEGS_WAVE) + wave));
         u < nunits; u += nw) {
        const UnitCtx c = udesc[u];
        const uint32_t o = lane < SUPER_TILES ? ucnt[(int64_t)u * SUPER_TILES + lane] : 0u;
        uint32_t m[NQ];
        uint2 gd[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const uint32_t e = c.e0 + q * LEGS_WAVE + lane;
            m[q] = 0;
            gd[q] = make_uint2(0u, 0u);
            if (e < c.e1) {
                const uint32_t pos = clist[e];
                if ((int64_t)pos < G) {
                    const FRec r = pay[e];
                    m[q] = entry_mask(pos, r, c, cpos, ckeep);
                    gd[q] = make_uint2(r.gid, r.dbits);
                }
            }
        }
        const int64_t tbase = c.toff + (int64_t)c.ty0 * c.tiles_x + c.tx0;
        for (int b0 = 0; b0 < SUPER_TILES; b0 += TB) {
            uint32_t tot[TB];
#pragma unroll
            for (int bb = 0; bb < TB; ++bb) {
                const int b = b0 + bb;
                tot[bb] = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                    const uint64_t bal = legs_ballot((m[q] >> b) & 1u);
                    if ((m[q] >> b) & 1u)
                        run[bb][tot[bb] + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u))] =
                            gd[q];
                    tot[bb] += (uint32_t)__popcll(bal);
                }
            }
#pragma unroll
            for (int bb = 0; bb < TB; ++bb) {
                if (tot[bb] == 0) continue;
                const int b = b0 + bb;
                const uint32_t start = (uint32_t)__builtin_amdgcn_readlane((int)o, b);
                const uint64_t tile = (uint64_t)(tbase + (int64_t)(b / SX) * c.tiles_x + b % SX);
                for (uint32_t k = lane; k < tot[bb]; k += LEGS_WAVE) {
                    const uint2 v = run[bb][k];
                    const int64_t at = (int64_t)start + k;
                    if (at < capacity) {
                        if (keys) keys[at] = (tile << 32) | v.y;
                        ids[at] = v.x;
                    }
                }
            }
        }
    }
}

// ---- tile ranges --------------------------------------------------------------

__global__ void __launch_bounds__(256)
k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

__global__ void __launch_bounds__(256)
k_ranges(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ count, int64_t capacity,
         uint32_t *__restrict__ ranges)
{
    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
        const uint32_t t = (uint32_t)(keys[i] >> 32);
        if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != t) ranges[2 * (int64_t)t] = (uint32_t)i;
        if (i == m - 1 || (uint32_t)(keys[i + 1] >> 32) != t) ranges[2 * (int64_t)t + 1] = (uint32_t)(i + 1);
    }
}

} // namespace

legs_sort_layout legs_sort_layout_for(int64_t capacity, int64_t total_tiles)
{
    auto up = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
    legs_sort_layout L;
    const int64_t parts = (capacity + LEGS_SORT_PART - 1) / LEGS_SORT_PART;
    L.parts = parts > 0 ? parts : 1;
    L.hist_off = 0;
    L.counter_off = L.hist_off + 4 * LEGS_SORT_MAX_PASSES * 256;
    L.status_off = L.counter_off + 256;  // 64 counters
    int64_t o = up(L.status_off + 8 * (int64_t)LEGS_SORT_MAX_PASSES * L.parts * 256);
    const int64_t T = total_tiles > 0 ? total_tiles : 0;   // the G-view sort needs none of these
    L.ccap = T > 0 ? capacity + T : 0;
    const int64_t units = T > 0 ? L.ccap / LEGS_COMPACT_UNIT + T : 0;
    L.tcount_off = o; o = up(o + 4 * T);
    L.scount_off = o; o = up(o + 4 * T);     // right after tcount: both are cleared at once
    L.cranges_off = o; o = up(o + 8 * T);
    L.uoff_off = o; o = up(o + 4 * (T + 1));
    L.desc_off = o; o = up(o + 256);
    L.clist_off = o; o = up(o + 16 * L.ccap);
    L.ucnt_off = o; o = up(o + 4 * 32 * units);
    L.udesc_off = o; o = up(o + 32 * units);
    L.cpay_off = o; o = up(o + 16 * L.ccap);
    L.part_off = o; o = up(o + 4 * (int64_t)LEGS_TILE_CHUNKS * T);
    L.spart_off = o; o = up(o + 4 * (int64_t)LEGS_TILE_CHUNKS * T);
    L.seg_off = o; o = up(o + (T > 0 ? 2 * 4 * (int64_t)LEGS_SEG_MAX * 256 : 0));
    L.order_off = o; o = up(o + 4 * T);
    L.total = o;
    return L;
}

static int grid_for(legs_ctx *ctx, int64_t work, int per_block, int waves_per_cu)
{
    int64_t b = (work + per_block - 1) / per_block;
    const int64_t cap = (int64_t)ctx->num_cus * waves_per_cu;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

namespace {

struct SortScratch {
    uint32_t *hist, *counters;
    uint64_t *status;
    int64_t parts;
    // depth-first binning
    int64_t ccap;
    uint32_t *tcount, *scount, *cranges, *uoff, *desc, *clist, *ucnt, *partial, *spartial, *seg_hist,
        *seg_off;
    uint64_t *cut;
    char *udesc, *cpay;
};

SortScratch sort_scratch_at(void *base, int64_t capacity, int64_t total_tiles = 0)
{
    const legs_sort_layout L = legs_sort_layout_for(capacity, total_tiles);
    char *b = static_cast<char *>(base);
    auto u32 = [b](int64_t off) { return reinterpret_cast<uint32_t *>(b + off); };
    auto u64 = [b](int64_t off) { return reinterpret_cast<uint64_t *>(b + off); };
    SortScratch S;
    S.hist = u32(L.hist_off);
    S.counters = u32(L.counter_off);
    S.status = u64(L.status_off);
    S.parts = L.parts;
    S.ccap = L.ccap;
    S.tcount = u32(L.tcount_off);
    S.scount = u32(L.scount_off);
    S.cranges = u32(L.cranges_off);
    S.uoff = u32(L.uoff_off);
    S.desc = u32(L.desc_off);
    S.cut = u64(L.desc_off + 128);
    S.clist = u32(L.clist_off);
    S.ucnt = u32(L.ucnt_off);
    S.udesc = b + L.udesc_off;
    S.cpay = b + L.cpay_off;
    S.partial = u32(L.part_off);
    S.spartial = u32(L.spart_off);
    S.seg_hist = u32(L.seg_off);
    S.seg_off = S.seg_hist + (int64_t)LEGS_SEG_MAX * 256;
    return S;
}

// LSD onesweep passes over digits [first, last) of (key, value) pairs; the
// input is in (k0, v0) and the buffers ping-pong, so the result ends in
// (k0, v0) when last - first is even and in (k1, v1) otherwise. Unless
// prepared, the scratch is cleared and the digits counted here first.
int32_t radix_passes(legs_ctx *ctx, const SortScratch &S, uint64_t *k0, uint32_t *v0,
                     uint64_t *k1, uint32_t *v1, const uint64_t *count, int64_t capacity,
                     int first, int last, bool prepared, hipStream_t s, int shift0 = 0)
{
    const int np = last - first;
    if (np <= 0) return LEGS_OK;
    if (!prepared) {   // prepared: the caller cleared the scratch and counted the digits
        const int gclear = grid_for(ctx, S.parts * 256 * np, 256, 8);
        hipLaunchKernelGGL(k_sort_clear, dim3(gclear), dim3(256), 0, s,
                           SortClearArgs{S.status, S.parts, np, S.counters, S.hist, count, capacity});
        const int ghist = grid_for(ctx, capacity, 256 * HIST_RUN, 4);
        hipLaunchKernelGGL(k_histogram, dim3(ghist), dim3(256), 0, s, k0, count, capacity, first, np, S.hist);
        LEGS_CHECK_LAUNCH(ctx);
    }
    const int gsort = grid_for(ctx, capacity, LEGS_SORT_PART, 2);
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (int p = first; p < last; ++p) {
        hipLaunchKernelGGL((k_onesweep<uint64_t, false>), dim3(gsort), dim3(LEGS_SORT_THREADS), 0, s,
                           ka, va, kb, vb, count, capacity, p, shift0 + 8 * p, 8, nullptr, S.hist,
                           S.status + (int64_t)(p - first) * S.parts * 256, S.counters + (p - first),
                           CoarsePay{}, nullptr);
        LEGS_CHECK_LAUNCH(ctx);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    return LEGS_OK;
}

struct OrderLayout {
    int64_t G, nbs;
    int64_t k0, k1, v0, v1, bcounts, offsets, cbcounts, coffsets, gcount, ccount, frecs, crecs, vrange,
        sviews, sort, total;
};

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

OrderLayout order_layout(int64_t n, int32_t n_views)
{
    OrderLayout L;
    L.G = n * (int64_t)n_views;
    L.nbs = (L.G + LEGS_PROJ_BLOCK - 1) / LEGS_PROJ_BLOCK;
    int64_t o = 0;
    L.k0 = o; o = align256(o + 8 * L.G);
    L.k1 = o; o = align256(o + 8 * L.G);
    L.v0 = o; o = align256(o + 4 * L.G);
    L.v1 = o; o = align256(o + 4 * L.G);
    L.bcounts = o; o = align256(o + 8 * (L.nbs + 1));
    L.offsets = o; o = align256(o + 8 * (L.nbs + 1));
    L.cbcounts = o; o = align256(o + 8 * (L.nbs + 1));
    L.coffsets = o; o = align256(o + 8 * (L.nbs + 1));
    L.gcount = o; o = align256(o + 8);
    L.ccount = o; o = align256(o + 8);
    L.frecs = o; o = align256(o + 16 * L.G);
    L.crecs = o; o = align256(o + 16 * L.G);
    L.vrange = o; o = align256(o + 16 * (int64_t)n_views);
    L.sviews = o; o = align256(o + (int64_t)sizeof(legs_view) * n_views);
    L.sort = o; o = align256(o + legs_sort_layout_for(L.G).total);
    L.total = o;
    return L;
}

int bits_for(int64_t count)
{
    int b = 0;
    while (b < 32 && (1ll << b) < count) ++b;
    return b;
}

} // namespace

int64_t legs_order_scratch_bytes(int64_t n, int32_t n_views) { return order_layout(n, n_views).total; }

int32_t legs_launch_bin_sort(legs_ctx *ctx, const legs_projected *proj, int64_t n,
                             const legs_view *views, int32_t n_views, int64_t total_tiles,
                             const legs_opts *o, legs_bins *bins, int64_t *host_count,
                             hipStream_t s)
{
    const int passes = legs_sort_passes(total_tiles);
    const bool full = (o->flags & LEGS_FLAG_FULL_SORT) != 0 || !proj->order;
    if (!full && bins->capacity + total_tiles >= (1ll << 32))
        return legs_set_error(ctx, LEGS_ERR_ARG,
                              "legs_bin_sort: capacity + total_tiles must be below 2^32 for the "
                              "depth-first binning (LEGS_FLAG_FULL_SORT lifts this)");
    const SortScratch S = sort_scratch_at(bins->scratch, bins->capacity, full ? 0 : total_tiles);
    uint64_t *offsets = nullptr, *coffsets = nullptr, *ccount = nullptr;
    const uint32_t *perm = nullptr;
    int64_t nblocks = 0;
    char *ord = static_cast<char *>(proj->order);
    OrderLayout OL;
    legs_view *sviews = nullptr;
    if (!full) {
        // 1. depth order of every visible G-view: the four depth-digit passes of
        //    the key sort, run once per Gaussian instead of once per instance
        OL = order_layout(n, n_views);
        uint64_t *ok0 = reinterpret_cast<uint64_t *>(ord + OL.k0), *ok1 = reinterpret_cast<uint64_t *>(ord + OL.k1);
        uint32_t *ov0 = reinterpret_cast<uint32_t *>(ord + OL.v0), *ov1 = reinterpret_cast<uint32_t *>(ord + OL.v1);
        uint64_t *gcount = reinterpret_cast<uint64_t *>(ord + OL.gcount);
        const int gpass = (32 + bits_for(n_views) + 7) / 8;
        // the G-view index in the key's low bits when the digits still fit in
        // 64 bits: the passes move 8 bytes per G-view instead of 12
        const int vb = bits_for(OL.G);
        const int vbits = (vb > 0 && vb + 8 * gpass <= 64) ? vb : 0;
        uint64_t *vrange = reinterpret_cast<uint64_t *>(ord + OL.vrange);
        sviews = reinterpret_cast<legs_view *>(ord + OL.sviews);
        {
            // one set-up launch: the G-view sort scratch cleared for every G-view,
            // the super-tile views, and the clears of the counting and coarse
            // scratch (both grids' cell counts are adjacent)
            const SortScratch GS = sort_scratch_at(ord + OL.sort, OL.G);
            const SortClearArgs ca = OL.G > 0 ? SortClearArgs{GS.status, GS.parts, gpass, GS.counters, GS.hist,
                                                              nullptr, OL.G}
                                              : SortClearArgs{nullptr, 0, 0, nullptr, nullptr, nullptr, 0};
            const int64_t nclear = (int64_t)(S.scount - S.tcount) + total_tiles;
            const SuperViewArgs sa{views, n_views, sviews, S.desc, S.hist, S.counters, S.cut, vrange, S.tcount,
                                   nclear};
            const int g0 = OL.G > 0 ? grid_for(ctx, GS.parts * 256 * gpass, 256, 8) : 1;
            const int g1 = grid_for(ctx, nclear, 256, 8);
            hipLaunchKernelGGL(k_bin_setup, dim3(g0 > g1 ? g0 : g1), dim3(256), 0, s, ca, sa);
        }
        if (OL.G > 0) {
            // the keys with their digit counts, then the passes
            const SortScratch GS = sort_scratch_at(ord + OL.sort, OL.G);
            hipLaunchKernelGGL(k_order_keys, dim3(grid_for(ctx, OL.G, ORDER_THREADS * ORDER_RUN, 4)),
                               dim3(ORDER_THREADS), 0, s,
                               proj->ntiles, proj->depth, n, OL.G, ok0, ov0, gcount, gpass, GS.hist, vbits);
            LEGS_CHECK_LAUNCH(ctx);
            const int32_t r = vbits > 0
                                  ? radix_passes(ctx, GS, ok0, nullptr, ok1, nullptr, gcount, OL.G, 0, gpass, true, s,
                                                 vbits)
                                  : radix_passes(ctx, GS, ok0, ov0, ok1, ov1, gcount, OL.G, 0, gpass, true, s);
            if (r != LEGS_OK) return r;
        }
        perm = vbits > 0 ? nullptr : (gpass % 2 == 0) ? ov0 : ov1;
        nblocks = OL.nbs;
        uint64_t *bcounts = reinterpret_cast<uint64_t *>(ord + OL.bcounts);
        uint64_t *cbcounts = reinterpret_cast<uint64_t *>(ord + OL.cbcounts);
        offsets = reinterpret_cast<uint64_t *>(ord + OL.offsets);
        coffsets = reinterpret_cast<uint64_t *>(ord + OL.coffsets);
        ccount = reinterpret_cast<uint64_t *>(ord + OL.ccount);
        if (nblocks > 0)
            hipLaunchKernelGGL(k_sorted_records, dim3((unsigned)nblocks), dim3(LEGS_PROJ_BLOCK), 0, s,
                               perm, (gpass % 2 == 0) ? ok0 : ok1, vbits,
                               reinterpret_cast<const int4 *>(proj->box), n, OL.G, sviews, o->tile,
                               reinterpret_cast<FRec *>(ord + OL.frecs),
                               reinterpret_cast<GRec *>(ord + OL.crecs), vrange, bcounts, cbcounts);
        hipLaunchKernelGGL(k_scan_pair, dim3(2), dim3(1024), 0, s, ScanArgs{bcounts, offsets, nblocks, bins->count},
                           ScanArgs{cbcounts, coffsets, nblocks, ccount});
    } else {
        // 1'. instance offsets in Gaussian order from the projection's block counts
        nblocks = ((n + LEGS_PROJ_BLOCK - 1) / LEGS_PROJ_BLOCK) * n_views;
        offsets = proj->block_offsets + nblocks + 1;
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, proj->block_offsets, offsets,
                           nblocks, bins->count);
    }
    LEGS_CHECK_LAUNCH(ctx);
    if (host_count) {
        uint64_t tot = 0;
        LEGS_CHECK_HIP(ctx, hipMemcpyAsync(&tot, bins->count, sizeof(tot), hipMemcpyDeviceToHost, s));
        LEGS_CHECK_HIP(ctx, hipStreamSynchronize(s));
        *host_count = (int64_t)tot;
        if ((int64_t)tot > bins->capacity)
            return legs_set_error(ctx, LEGS_ERR_CAPACITY,
                                  "legs_bin_sort: %lld instances exceed capacity %lld",
                                  (long long)tot, (long long)bins->capacity);
    }
    if (full) {
        // 2'. emission in Gaussian order, all eight digit passes over the
        //     instances, ranges from the sorted keys
        const int np = passes;
        uint64_t *k0 = (np % 2 == 0) ? bins->keys : bins->keys_alt;
        uint32_t *v0 = (np % 2 == 0) ? bins->ids : bins->ids_alt;
        uint64_t *k1 = (np % 2 == 0) ? bins->keys_alt : bins->keys;
        uint32_t *v1 = (np % 2 == 0) ? bins->ids_alt : bins->ids;
        if (n > 0 && n_views > 0) {
            const int64_t bx = (n + LEGS_PROJ_BLOCK - 1) / LEGS_PROJ_BLOCK;
            hipLaunchKernelGGL(k_emit, dim3((unsigned)bx, (unsigned)n_views), dim3(LEGS_PROJ_BLOCK), 0, s,
                               reinterpret_cast<const int4 *>(proj->box), proj->depth, proj->ntiles,
                               offsets, n, views, o->tile, bins->capacity, k0, v0);
            LEGS_CHECK_LAUNCH(ctx);
        }
        const int32_t r = radix_passes(ctx, S, k0, v0, k1, v1, bins->count, bins->capacity, 0,
                                       passes, false, s);
        if (r != LEGS_OK) return r;
        const int gfill = grid_for(ctx, 2 * total_tiles, 256, 8);
        hipLaunchKernelGGL(k_fill_u32, dim3(gfill), dim3(256), 0, s, bins->ranges, 2 * total_tiles, 0u);
        LEGS_CHECK_LAUNCH(ctx);
        const int grng = grid_for(ctx, bins->capacity, 256, 16);
        hipLaunchKernelGGL(k_ranges, dim3(grng), dim3(256), 0, s, bins->keys, bins->count,
                           bins->capacity, bins->ranges);
        LEGS_CHECK_LAUNCH(ctx);
        return LEGS_OK;
    }

    const FRec *frecs = reinterpret_cast<const FRec *>(ord + OL.frecs);
    const GRec *crecs = reinterpret_cast<const GRec *>(ord + OL.crecs);
    const uint64_t *vrange = reinterpret_cast<const uint64_t *>(ord + OL.vrange);
    const int64_t T = total_tiles;
    // enough workgroups per view to spread the G-views, at most LEGS_TILE_CHUNKS
    int nch = (int)(((OL.G / (n_views > 0 ? n_views : 1)) + 4095) / 4096);
    nch = nch < 1 ? 1 : (nch > LEGS_TILE_CHUNKS ? LEGS_TILE_CHUNKS : nch);

    // 2. per-cell counts of the tile stream (cut at the capacity) and of the
    //    coarse stream (every G-view's super-tile rectangle, cut at the coarse
    //    capacity, which holds every G-view the tile stream keeps): the tile
    //    ranges, the super-tile list ranges, the digit histograms of the coarse
    //    passes, and the G-view the tile cut falls in
    CountGrid cg0{views, S.tcount, S.partial, bins->ranges, nullptr, nullptr};
    CountGrid cg1{sviews, S.scount, S.spartial, S.cranges, S.desc, S.hist};
    hipLaunchKernelGGL(k_count_corners, dim3((unsigned)nch, (unsigned)n_views), dim3(256), 0, s, frecs, crecs,
                       offsets, coffsets, vrange, OL.G, bins->capacity, S.ccap, T, bins->count, ccount, cg0, cg1,
                       S.cut);
    hipLaunchKernelGGL(k_count_merge, dim3((unsigned)((2 * T + 255) / 256), 32), dim3(256), 0, s, nch, T, n_views,
                       cg0, cg1);
    hipLaunchKernelGGL(k_count_prefix, dim3((unsigned)n_views, 2), dim3(1024), 0, s, cg0, cg1);
    hipLaunchKernelGGL(k_count_lists, dim3(3), dim3(1024), 0, s, T, cg0, cg1, S.uoff);
    LEGS_CHECK_LAUNCH(ctx);
    // passes for the most super-tiles there can be (one per tile); the ones
    // the actual count does not need return at once
    const int cpasses = (bits_for(T) + 7) / 8 > 0 ? (bits_for(T) + 7) / 8 : 1;

    // 4. coarse passes: the (super-tile, position) pairs written out in stream
    //    order, then stable counting passes over the super-tile digits; pass p
    //    reads buffer 1 - p % 2 and writes buffer p % 2, and the last one also
    //    writes the tile record of each entry
    uint32_t *ck[2] = {S.clist, S.clist + S.ccap};
    uint32_t *cv[2] = {S.clist + 2 * S.ccap, S.clist + 3 * S.ccap};
    if (nblocks > 0)
        hipLaunchKernelGGL(k_coarse_emit, dim3((unsigned)nblocks), dim3(LEGS_PROJ_BLOCK), 0, s, crecs, coffsets,
                           OL.G, S.ccap, ck[1], cv[1]);
    const CoarsePay P{frecs, reinterpret_cast<FRec *>(S.cpay), OL.G};
    // one partition per segment up to LEGS_SEG_MAX segments (segments past the
    // last partition return at once)
    const int nseg = LEGS_SEG_MAX;
    for (int p = 0; p < cpasses; ++p) {
        const int wo = p % 2, ri = 1 - wo;
        hipLaunchKernelGGL(k_coarse_upsweep, dim3(nseg), dim3(LEGS_SORT_THREADS), 0, s, ck[ri], ccount, S.ccap,
                           S.desc, p, S.seg_hist);
        hipLaunchKernelGGL(k_seg_scan, dim3(256), dim3(LEGS_SEG_MAX), 0, s, S.seg_hist, nseg, S.hist, S.desc,
                           p, S.seg_off);
        hipLaunchKernelGGL((k_onesweep<uint32_t, true>), dim3(nseg), dim3(LEGS_SORT_THREADS), 0, s, ck[ri], cv[ri],
                           ck[wo], cv[wo], ccount, S.ccap, p, 0, 0, S.desc, nullptr, nullptr, nullptr, P,
                           S.seg_off);
        LEGS_CHECK_LAUNCH(ctx);
    }

    // 5. compaction of the super-tile lists into the tile lists, in units of
    //    LEGS_COMPACT_UNIT list entries per wave
    const int64_t max_units = S.ccap / LEGS_COMPACT_UNIT + T;
    const int gu = grid_for(ctx, max_units, 256 / LEGS_WAVE, 8);
    UnitCtx *udesc = reinterpret_cast<UnitCtx *>(S.udesc);
    hipLaunchKernelGGL(k_unit_desc, dim3(grid_for(ctx, max_units, 256, 4)), dim3(256), 0, s, S.uoff, T, S.cranges,
                       sviews, views, n_views, udesc);
    hipLaunchKernelGGL(k_compact_count, dim3(gu), dim3(256), 0, s, cv[0], cv[1], S.desc, S.uoff, T, udesc, P.pay,
                       OL.G, S.cut, S.ucnt);
    hipLaunchKernelGGL(k_compact_scan, dim3(grid_for(ctx, T, 256 / LEGS_WAVE, 4)), dim3(256), 0, s, S.uoff, T,
                       sviews, views, n_views, bins->ranges, S.ucnt);
    hipLaunchKernelGGL(k_compact_write, dim3(gu), dim3(256), 0, s, cv[0], cv[1], S.desc, S.uoff, T, udesc, P.pay,
                       OL.G, S.cut, S.ucnt, bins->capacity,
                       (o->flags & LEGS_FLAG_IDS_ONLY) ? nullptr : bins->keys, bins->ids);
    LEGS_CHECK_LAUNCH(ctx);
    return LEGS_OK;
}
