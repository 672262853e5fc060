// Tile binning for the rasteriser (gfx950): instance scan, key emission, a
// stable LSD onesweep radix sort of 64-bit (tile << 32 | depth bits) keys with
// 32-bit Gaussian ids, and per-tile [start, end) ranges.
//
// Every kernel after the scan reads the instance count from device memory and
// walks it with a fixed grid, so the whole chain can be captured in a HIP
// graph without knowing the count on the host.
//
// Onesweep (one pass per 8-bit digit): digit histograms for every pass come
// from one upfront read of the keys; each pass then ranks a 4096-key
// partition per workgroup with wave64 ballots (stable: ties keep input order),
// publishes per-digit partition counts, and resolves its global offsets by
// decoupled look-back over earlier partitions. Partition ids are handed out
// by an atomic counter in launch order, so every partition a workgroup waits
// on belongs to a workgroup that is already running (forward progress without
// relying on blockIdx scheduling order). Keys are first scattered into LDS in
// digit order, then written out so consecutive lanes write consecutive
// addresses within a digit run.
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

// One workgroup: exclusive scan of counts[0..nb) into offsets[0..nb], total
// in offsets[nb] and in *total (counts stay intact, so the binning can rerun).
__global__ void __launch_bounds__(1024)
k_scan_blocks(const uint64_t *__restrict__ counts, uint64_t *__restrict__ offsets, int64_t nb,
              uint64_t *__restrict__ total)
{
    __shared__ uint64_t s_w[16];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const uint64_t x = i < nb ? counts[i] : 0;
        uint64_t incl = x;
#pragma unroll
        for (int off = 1; off < LEGS_WAVE; off <<= 1) {
            const uint64_t y = __shfl_up(incl, off, LEGS_WAVE);
            if (lane >= off) incl += y;
        }
        if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
        __syncthreads();
        uint64_t wpre = 0;
        for (int w = 0; w < wave; ++w) wpre += s_w[w];
        const uint64_t carry = s_carry;
        if (i < nb) offsets[i] = carry + wpre + incl - x;
        __syncthreads();
        if (threadIdx.x == 1023) s_carry = carry + wpre + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        offsets[nb] = s_carry;
        *total = s_carry;
    }
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

// Digit histograms of passes [first, first + npass) in one read of the keys.
// Loads are coalesced (lane l reads key base + 64 i + l); within each wave a
// run of equal digits in consecutive lanes is counted with one LDS atomic by
// its first lane (run starts from a ballot). Instance keys come in long runs
// (every tile of one Gaussian shares its depth digits, consecutive tiles of a
// row share the high tile digits), so hot digits no longer serialise.
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

// Exclusive scan of each pass's 256 digit counts (one workgroup per pass).
__global__ void __launch_bounds__(256)
k_digit_starts(const uint32_t *__restrict__ hist, uint32_t *__restrict__ starts, int first)
{
    const int p = first + blockIdx.x, d = threadIdx.x;
    const int lane = legs_lane(), wave = d / LEGS_WAVE;
    const uint32_t x = hist[p * 256 + d];
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    __shared__ uint32_t s_w[4];
    if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += s_w[w];
    starts[p * 256 + d] = pre + incl - x;
}

// Zero the look-back status words of every pass and the partition counters,
// only as far as the partitions this count needs.
__global__ void __launch_bounds__(256)
k_sort_clear(uint64_t *__restrict__ status, int64_t parts_cap, int passes,
             uint32_t *__restrict__ counters, uint32_t *__restrict__ hist,
             const uint64_t *__restrict__ count, int64_t capacity)
{
    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    const int64_t parts = (m + LEGS_SORT_PART - 1) / LEGS_SORT_PART;
    const int64_t per_pass = parts * 256;
    const int64_t tot = per_pass * passes;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += stride) {
        const int64_t p = i / per_pass, r = i - p * per_pass;
        status[p * parts_cap * 256 + r] = 0;
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x < 16) counters[threadIdx.x] = 0;
        for (int i = threadIdx.x; i < LEGS_SORT_MAX_PASSES * 256; i += 256) hist[i] = 0;
    }
}

// Inputs of the fused emission (first tile pass of the depth-first binning):
// the depth-ordered G-views and the instance offset of every 256 of them.
struct TileEmit {
    const uint32_t *perm;      // G-view index at each depth-ordered position
    const int4 *box;
    const uint32_t *ntiles;
    const uint64_t *goff;      // [nblocks + 1] instance offset of each block of 256 positions
    int64_t nblocks, n, G;
    const legs_view *views;
    int tile;
};

// Output of the last tile pass: the 64-bit keys (tile << 32) | bits(depth).
struct TileFinal {
    uint64_t *keys64;
    const float *depth;
    int64_t n;
    const legs_view *views;
    int n_views;
};

// Exclusive scan of one value per thread over a 256-thread block (64-bit
// totals); s_start[256] receives the block total.
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
    uint64_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += s_w[w];
    s_start[threadIdx.x] = wpre + incl - x;
    if (threadIdx.x == 255) s_start[256] = wpre + incl;
    __syncthreads();
}

// One onesweep pass over digit `pass` (bits 8 pass .. 8 pass + 7) of keys K.
// EMIT: the partition's (tile, id) pairs are generated from the depth-ordered
// G-views instead of read (instance e of the stream is tile e - start of its
// G-view's rectangle, row-major). FINAL: the output keys are widened to the
// 64-bit (tile << 32) | bits(depth) keys of the tile lists.
template <typename K, bool EMIT, bool FINAL>
__global__ void __launch_bounds__(LEGS_SORT_THREADS)
k_onesweep(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
           K *__restrict__ kout, uint32_t *__restrict__ vout,
           const uint64_t *__restrict__ count, int64_t capacity, int pass,
           const uint32_t *__restrict__ digit_starts, uint64_t *__restrict__ status,
           uint32_t *__restrict__ counter, TileEmit E, TileFinal F)
{
    constexpr int NW = LEGS_SORT_THREADS / LEGS_WAVE;
    static_assert(LEGS_SORT_THREADS == 256, "one thread per digit");
    __shared__ K s_keys[LEGS_SORT_PART];
    __shared__ uint32_t s_vals[LEGS_SORT_PART];
    __shared__ uint32_t s_wh[NW][256];      // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_lstart[256];      // block-local start of each digit
    __shared__ uint64_t s_gstart[257];      // global start of this partition's digit runs;
                                            // with EMIT first the G-view scan of a block
    __shared__ uint32_t s_tmp[NW];
    __shared__ uint64_t s_w64[NW];
    __shared__ int64_t s_part;

    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    const int64_t parts = (m + LEGS_SORT_PART - 1) / LEGS_SORT_PART;
    const int shift = 8 * pass;
    const int tid = threadIdx.x, lane = legs_lane(), wave = tid / LEGS_WAVE;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    for (;;) {
        if (tid == 0) s_part = (int64_t)atomicAdd(counter, 1u);
        for (int i = tid; i < NW * 256; i += LEGS_SORT_THREADS) (&s_wh[0][0])[i] = 0;
        __syncthreads();
        const int64_t part = s_part;
        if (part >= parts) break;
        const int64_t base = part * LEGS_SORT_PART;
        const int64_t nvalid64 = m - base < LEGS_SORT_PART ? m - base : LEGS_SORT_PART;
        const int nvalid = (int)nvalid64;

        if constexpr (EMIT) {
            // first block of G-views whose instances reach this partition
            __shared__ int64_t s_b;
            if (tid == 0) {
                int64_t lo = 0, hi = E.nblocks - 1;
                while (lo < hi) {
                    const int64_t mid = (lo + hi + 1) >> 1;
                    if (E.goff[mid] <= (uint64_t)base) lo = mid; else hi = mid - 1;
                }
                s_b = lo;
            }
            __syncthreads();
            __shared__ int s_tx0[256], s_ty0[256], s_rw[256], s_tilesx[256];
            __shared__ int64_t s_toff[256];
            __shared__ uint32_t s_g[256];
            for (int64_t b = s_b; b < E.nblocks; ++b) {
                const uint64_t ob = E.goff[b];
                if (ob >= (uint64_t)(base + nvalid)) break;
                const int64_t pos = b * 256 + tid;
                uint64_t c = 0;
                if (pos < E.G) {
                    const int64_t gv = E.perm[pos];
                    c = E.ntiles[gv];
                    if (c) {
                        const int64_t v = gv / E.n;
                        const int4 bx = E.box[gv];
                        s_tx0[tid] = bx.x / E.tile;
                        s_ty0[tid] = bx.z / E.tile;
                        s_rw[tid] = bx.y / E.tile - bx.x / E.tile + 1;
                        s_g[tid] = (uint32_t)(gv - v * E.n);
                        s_toff[tid] = E.views[v].tile_offset;
                        s_tilesx[tid] = E.views[v].tiles_x;
                    }
                }
                block_scan_256(c, s_gstart, s_w64);
                const uint64_t tot = s_gstart[256];
                const uint64_t lo = (uint64_t)base > ob ? (uint64_t)base - ob : 0;
                const uint64_t hi = ((uint64_t)(base + nvalid) - ob) < tot ? (uint64_t)(base + nvalid) - ob : tot;
                for (uint64_t k = lo + tid; k < hi; k += LEGS_SORT_THREADS) {
                    int l0 = 0, l1 = 255;
                    while (l0 < l1) {
                        const int mid = (l0 + l1 + 1) >> 1;
                        if (s_gstart[mid] <= k) l0 = mid; else l1 = mid - 1;
                    }
                    const uint32_t local = (uint32_t)(k - s_gstart[l0]);
                    const int rw = s_rw[l0];
                    const int ty = s_ty0[l0] + (int)(local / (uint32_t)rw);
                    const int tx = s_tx0[l0] + (int)(local % (uint32_t)rw);
                    const int64_t e = (int64_t)(ob + k) - base;
                    s_keys[e] = (K)(s_toff[l0] + (int64_t)ty * s_tilesx[l0] + tx);
                    s_vals[e] = s_g[l0];
                }
                __syncthreads();
            }
        }

        K key[LEGS_SORT_ITEMS];
        uint32_t val[LEGS_SORT_ITEMS];
        uint32_t rank[LEGS_SORT_ITEMS];
        // wave-striped: item i of lane l of wave w is partition element w*64*ITEMS + i*64 + l
#pragma unroll
        for (int i = 0; i < LEGS_SORT_ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * LEGS_SORT_ITEMS + i * LEGS_WAVE + lane;
            if (e < nvalid) {
                if constexpr (EMIT) { key[i] = s_keys[e]; val[i] = s_vals[e]; }
                else { key[i] = kin[base + e]; val[i] = vin[base + e]; }
            } else {
                key[i] = (K)~(K)0;
                val[i] = 0;
            }
        }
        if constexpr (EMIT) __syncthreads();   // s_keys is reused by the scatter below
        // rank within the wave: peers with the same digit via 8 ballots
#pragma unroll
        for (int i = 0; i < LEGS_SORT_ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * LEGS_SORT_ITEMS + i * LEGS_WAVE + lane;
            const bool ok = e < nvalid;
            const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
            uint64_t peers = legs_ballot(ok);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t bal = legs_ballot((d >> b) & 1u);
                peers &= ((d >> b) & 1u) ? bal : ~bal;
            }
            // the lowest peer reserves the run for all of them; an LDS atomic keeps
            // the reservation ordered against the next item's reservation
            const int leader = ok ? __ffsll((unsigned long long)peers) - 1 : lane;
            uint32_t pre = 0;
            if (ok && lane == leader) pre = atomicAdd(&s_wh[wave][d], (uint32_t)__popcll(peers));
            const uint32_t lbase = (uint32_t)__shfl((int)pre, leader, LEGS_WAVE);
            rank[i] = lbase + (uint32_t)__popcll(peers & lt_mask);
        }
        __syncthreads();
        // per digit: offsets of each wave, block total, look-back
        {
            const int d = tid;
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const uint32_t c = s_wh[w][d];
                s_wh[w][d] = t;
                t += c;
            }
            uint64_t *st = status + part * 256 + d;
            if (part == 0) st_status(st, FLAG_INC | (uint64_t)t);
            else st_status(st, FLAG_AGG | (uint64_t)t);
            uint64_t excl = 0;
            if (part > 0) {
                int64_t j = part - 1;
                for (;;) {
                    const uint64_t sv = ld_status(status + j * 256 + d);
                    const uint64_t f = sv & ~VALUE_MASK;
                    if (f == 0) continue;            // not published yet
                    excl += sv & VALUE_MASK;
                    if (f == FLAG_INC) break;
                    --j;
                }
                st_status(st, FLAG_INC | (excl + t));
            }
            s_gstart[d] = (uint64_t)digit_starts[pass * 256 + d] + excl;
            // block-local exclusive scan of digit totals
            uint32_t incl = t;
#pragma unroll
            for (int off = 1; off < LEGS_WAVE; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
                if (lane >= off) incl += y;
            }
            if (lane == LEGS_WAVE - 1) s_tmp[wave] = incl;
            __syncthreads();
            uint32_t wp = 0;
            for (int w = 0; w < wave; ++w) wp += s_tmp[w];
            s_lstart[d] = wp + incl - t;
        }
        __syncthreads();
        // scatter into LDS in digit order
#pragma unroll
        for (int i = 0; i < LEGS_SORT_ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * LEGS_SORT_ITEMS + i * LEGS_WAVE + lane;
            if (e < nvalid) {
                const uint32_t d = (uint32_t)(key[i] >> shift) & 255u;
                const uint32_t pos = s_lstart[d] + s_wh[wave][d] + rank[i];
                s_keys[pos] = key[i];
                s_vals[pos] = val[i];
            }
        }
        __syncthreads();
        // write out digit runs (positions past the capacity cannot occur when the
        // digit histograms count exactly the stored instances; the test keeps a
        // wrong histogram from writing out of bounds)
        for (int k = tid; k < nvalid; k += LEGS_SORT_THREADS) {
            const K kk = s_keys[k];
            const uint32_t d = (uint32_t)(kk >> shift) & 255u;
            const uint64_t gpos = s_gstart[d] + (uint64_t)(k - (int)s_lstart[d]);
            if (gpos >= (uint64_t)capacity) continue;
            if constexpr (FINAL) {
                const uint32_t id = s_vals[k];
                const int v = legs_view_of_tile(F.views, F.n_views, (int64_t)kk);
                F.keys64[gpos] = ((uint64_t)kk << 32) | __float_as_uint(F.depth[(int64_t)v * F.n + id]);
                vout[gpos] = id;
            } else {
                kout[gpos] = kk;
                vout[gpos] = s_vals[k];
            }
        }
        __syncthreads();
    }
}

// ---- depth order of the G-views ---------------------------------------------------

// key = (view << 32) | bits(depth) for visible G-views (culled ones sort last,
// they emit nothing); value = G-view index. Also stores G for the sort.
__global__ void __launch_bounds__(256)
k_order_keys(const uint32_t *__restrict__ ntiles, const float *__restrict__ depth, int64_t n,
             int64_t G, uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
             uint64_t *__restrict__ gcount)
{
    const int64_t gv = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (gv == 0) *gcount = (uint64_t)G;
    if (gv >= G) return;
    const uint64_t v = (uint64_t)(gv / n);
    keys[gv] = ntiles[gv] ? ((v << 32) | __float_as_uint(depth[gv])) : ~0ull;
    vals[gv] = (uint32_t)gv;
}

// Instance counts per block of 256 G-views in depth order.
__global__ void __launch_bounds__(LEGS_PROJ_BLOCK)
k_sorted_block_counts(const uint32_t *__restrict__ perm, const uint32_t *__restrict__ ntiles,
                      int64_t G, uint64_t *__restrict__ block_counts)
{
    const int64_t pos = (int64_t)blockIdx.x * LEGS_PROJ_BLOCK + threadIdx.x;
    uint64_t c = pos < G ? ntiles[perm[pos]] : 0u;
#pragma unroll
    for (int off = LEGS_WAVE / 2; off > 0; off >>= 1) c += __shfl_down(c, off, LEGS_WAVE);
    __shared__ uint64_t s_w[LEGS_PROJ_BLOCK / LEGS_WAVE];
    if (legs_lane() == 0) s_w[threadIdx.x / LEGS_WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < LEGS_PROJ_BLOCK / LEGS_WAVE; ++w) t += s_w[w];
        block_counts[blockIdx.x] = t;
    }
}

// ---- per-tile counts of the depth-ordered instance stream ----------------------

// The first `capacity` instances of the depth-ordered stream are counted per
// tile on a 2D difference array (the tile grid of each view): +1 / -1 at the
// corners of each G-view's tile rectangle, then prefix sums along the rows and
// the columns. A G-view cut by the capacity contributes its first tiles in
// row-major order (full rows plus one partial row). The counts give the
// tile ranges and the digit histograms of the tile passes without reading
// the instances.
__device__ __forceinline__ void diff_rect(uint32_t *diff, const legs_view &vw, int x0, int x1,
                                          int y0, int y1)
{
    uint32_t *g = diff + vw.tile_offset;
    const int W = vw.tiles_x, H = vw.tiles_y;
    atomicAdd(g + (int64_t)y0 * W + x0, 1u);
    if (x1 + 1 < W) atomicAdd(g + (int64_t)y0 * W + x1 + 1, 0xffffffffu);
    if (y1 + 1 < H) atomicAdd(g + (int64_t)(y1 + 1) * W + x0, 0xffffffffu);
    if (x1 + 1 < W && y1 + 1 < H) atomicAdd(g + (int64_t)(y1 + 1) * W + x1 + 1, 1u);
}

__global__ void __launch_bounds__(256)
k_tile_corners(const uint32_t *__restrict__ perm, const int4 *__restrict__ box,
               const uint32_t *__restrict__ ntiles, const uint64_t *__restrict__ goff, int64_t n,
               int64_t G, const legs_view *__restrict__ views, int tile, int64_t capacity,
               uint32_t *__restrict__ diff)
{
    __shared__ uint64_t s_start[257];
    __shared__ uint64_t s_w[4];
    const int64_t pos = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t gv = pos < G ? (int64_t)perm[pos] : 0;
    const uint64_t c = pos < G ? ntiles[gv] : 0u;
    block_scan_256(c, s_start, s_w);
    const uint64_t off = goff[blockIdx.x] + s_start[threadIdx.x];
    if (c == 0 || off >= (uint64_t)capacity) return;
    const uint64_t keep = (uint64_t)capacity - off < c ? (uint64_t)capacity - off : c;
    const int64_t v = gv / n;
    const legs_view vw = views[v];
    const int4 b = box[gv];
    const int x0 = b.x / tile, x1 = b.y / tile, y0 = b.z / tile, y1 = b.w / tile;
    if (keep == c) {
        diff_rect(diff, vw, x0, x1, y0, y1);
    } else {
        const int rw = x1 - x0 + 1;
        const int rows = (int)(keep / (uint64_t)rw), rem = (int)(keep % (uint64_t)rw);
        if (rows > 0) diff_rect(diff, vw, x0, x1, y0, y0 + rows - 1);
        if (rem > 0) diff_rect(diff, vw, x0, x0 + rem - 1, y0 + rows, y0 + rows);
    }
}

// Inclusive prefix sums along the tile rows of view blockIdx.y: one wave per row.
__global__ void __launch_bounds__(256)
k_tile_rows(uint32_t *__restrict__ diff, const legs_view *__restrict__ views)
{
    const legs_view vw = views[blockIdx.y];
    const int lane = legs_lane();
    const int row0 = blockIdx.x * 4 + (int)(threadIdx.x / LEGS_WAVE);
    for (int y = row0; y < vw.tiles_y; y += gridDim.x * 4) {
        uint32_t *r = diff + vw.tile_offset + (int64_t)y * vw.tiles_x;
        uint32_t carry = 0;
        for (int x0 = 0; x0 < vw.tiles_x; x0 += LEGS_WAVE) {
            const int x = x0 + lane;
            uint32_t incl = x < vw.tiles_x ? r[x] : 0u;
#pragma unroll
            for (int off = 1; off < LEGS_WAVE; off <<= 1) {
                const uint32_t t = __shfl_up(incl, off, LEGS_WAVE);
                if (lane >= off) incl += t;
            }
            if (x < vw.tiles_x) r[x] = carry + incl;
            carry += (uint32_t)__shfl((int)incl, LEGS_WAVE - 1, LEGS_WAVE);
        }
    }
}

// Inclusive prefix sums down the tile columns of view blockIdx.y: one lane per column.
__global__ void __launch_bounds__(256)
k_tile_cols(uint32_t *__restrict__ diff, const legs_view *__restrict__ views)
{
    const legs_view vw = views[blockIdx.y];
    for (int x = blockIdx.x * 256 + threadIdx.x; x < vw.tiles_x; x += gridDim.x * 256) {
        uint32_t *col = diff + vw.tile_offset + x;
        uint32_t acc = 0;
        for (int y = 0; y < vw.tiles_y; ++y) {
            acc += col[(int64_t)y * vw.tiles_x];
            col[(int64_t)y * vw.tiles_x] = acc;
        }
    }
}

// Sum of the tile counts of each block of 1024 tiles.
__global__ void __launch_bounds__(1024)
k_tile_block_sums(const uint32_t *__restrict__ counts, int64_t total_tiles, uint64_t *__restrict__ sums)
{
    __shared__ uint64_t s_w[16];
    const int64_t t = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint64_t x = t < total_tiles ? counts[t] : 0u;
#pragma unroll
    for (int off = LEGS_WAVE / 2; off > 0; off >>= 1) x += __shfl_down(x, off, LEGS_WAVE);
    if (legs_lane() == 0) s_w[threadIdx.x / LEGS_WAVE] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t s = 0;
        for (int w = 0; w < 16; ++w) s += s_w[w];
        sums[blockIdx.x] = s;
    }
}

// Tile ranges [start, start + count) from the scanned counts, and the digit
// histograms of the tile passes (digit p of a tile id counts its instances).
__global__ void __launch_bounds__(1024)
k_tile_ranges(const uint32_t *__restrict__ counts, int64_t total_tiles,
              const uint64_t *__restrict__ boff, int npass, uint32_t *__restrict__ ranges,
              uint32_t *__restrict__ hist)
{
    __shared__ uint32_t s_h[4][256];
    __shared__ uint64_t s_w[16];
    for (int i = threadIdx.x; i < 4 * 256; i += 1024) (&s_h[0][0])[i] = 0;
    const int lane = legs_lane(), wave = threadIdx.x / LEGS_WAVE;
    const int64_t t = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const uint64_t x = t < total_tiles ? counts[t] : 0u;
    uint64_t incl = x;
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint64_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
    __syncthreads();
    uint64_t wpre = 0;
    for (int w = 0; w < wave; ++w) wpre += s_w[w];
    if (t < total_tiles) {
        const uint64_t st = boff[blockIdx.x] + wpre + incl - x;
        ranges[2 * t] = (uint32_t)st;
        ranges[2 * t + 1] = (uint32_t)(st + x);
        if (x)
            for (int p = 0; p < npass; ++p) atomicAdd(&s_h[p][(uint32_t)(t >> (8 * p)) & 255u], (uint32_t)x);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < npass * 256; i += 1024) {
        const uint32_t c = (&s_h[0][0])[i];
        if (c) atomicAdd(&hist[i], c);
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
    legs_sort_layout L;
    const int64_t parts = (capacity + LEGS_SORT_PART - 1) / LEGS_SORT_PART;
    L.parts = parts > 0 ? parts : 1;
    L.hist_off = 0;
    L.start_off = L.hist_off + 4 * LEGS_SORT_MAX_PASSES * 256;
    L.counter_off = L.start_off + 4 * LEGS_SORT_MAX_PASSES * 256;
    L.status_off = L.counter_off + 256;  // 64 counters
    L.tcount_off = L.status_off + 8 * (int64_t)LEGS_SORT_MAX_PASSES * L.parts * 256;
    L.tile_blocks = (total_tiles + 1023) / 1024;
    L.tsum_off = (L.tcount_off + 4 * total_tiles + 255) & ~(int64_t)255;
    L.toff_off = L.tsum_off + 8 * (L.tile_blocks + 1);
    L.total = L.toff_off + 8 * (L.tile_blocks + 1) + 8;
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
    uint32_t *hist, *starts, *counters;
    uint64_t *status;
    int64_t parts;
    uint32_t *tcount;
    uint64_t *tsum, *toff;
    int64_t tile_blocks;
};

SortScratch sort_scratch_at(void *base, int64_t capacity, int64_t total_tiles = 0)
{
    const legs_sort_layout L = legs_sort_layout_for(capacity, total_tiles);
    char *b = static_cast<char *>(base);
    SortScratch S;
    S.hist = reinterpret_cast<uint32_t *>(b + L.hist_off);
    S.starts = reinterpret_cast<uint32_t *>(b + L.start_off);
    S.counters = reinterpret_cast<uint32_t *>(b + L.counter_off);
    S.status = reinterpret_cast<uint64_t *>(b + L.status_off);
    S.parts = L.parts;
    S.tcount = reinterpret_cast<uint32_t *>(b + L.tcount_off);
    S.tsum = reinterpret_cast<uint64_t *>(b + L.tsum_off);
    S.toff = reinterpret_cast<uint64_t *>(b + L.toff_off);
    S.tile_blocks = L.tile_blocks;
    return S;
}

// LSD onesweep passes over digits [first, last) of (key, value) pairs; the
// input is in (k0, v0) and the buffers ping-pong, so the result ends in
// (k0, v0) when last - first is even and in (k1, v1) otherwise.
int32_t radix_passes(legs_ctx *ctx, const SortScratch &S, uint64_t *k0, uint32_t *v0,
                     uint64_t *k1, uint32_t *v1, const uint64_t *count, int64_t capacity,
                     int first, int last, hipStream_t s)
{
    const int np = last - first;
    if (np <= 0) return LEGS_OK;
    const int gclear = grid_for(ctx, S.parts * 256 * np, 256, 8);
    hipLaunchKernelGGL(k_sort_clear, dim3(gclear), dim3(256), 0, s, S.status, S.parts, np,
                       S.counters, S.hist, count, capacity);
    const int ghist = grid_for(ctx, capacity, 256 * HIST_RUN, 4);
    hipLaunchKernelGGL(k_histogram, dim3(ghist), dim3(256), 0, s, k0, count, capacity, first, np,
                       S.hist);
    hipLaunchKernelGGL(k_digit_starts, dim3(np), dim3(256), 0, s, S.hist, S.starts, first);
    LEGS_CHECK_LAUNCH(ctx);
    const int gsort = grid_for(ctx, capacity, LEGS_SORT_PART, 2);
    uint64_t *ka = k0, *kb = k1;
    uint32_t *va = v0, *vb = v1;
    for (int p = first; p < last; ++p) {
        hipLaunchKernelGGL((k_onesweep<uint64_t, false, false>), dim3(gsort), dim3(LEGS_SORT_THREADS), 0, s,
                           ka, va, kb, vb, count, capacity, p, S.starts,
                           S.status + (int64_t)(p - first) * S.parts * 256, S.counters + (p - first),
                           TileEmit{}, TileFinal{});
        LEGS_CHECK_LAUNCH(ctx);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    return LEGS_OK;
}

struct OrderLayout {
    int64_t G, nbs;
    int64_t k0, k1, v0, v1, bcounts, offsets, gcount, sort, total;
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
    L.gcount = o; o = align256(o + 8);
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
    const SortScratch S = sort_scratch_at(bins->scratch, bins->capacity, full ? 0 : total_tiles);
    uint64_t *offsets = nullptr;
    const uint32_t *perm = nullptr;
    int64_t nblocks = 0;
    char *ord = static_cast<char *>(proj->order);
    OrderLayout OL;
    if (!full) {
        // 1. depth order of every visible G-view: the four depth-digit passes of
        //    the key sort, run once per Gaussian instead of once per instance
        OL = order_layout(n, n_views);
        uint64_t *ok0 = reinterpret_cast<uint64_t *>(ord + OL.k0), *ok1 = reinterpret_cast<uint64_t *>(ord + OL.k1);
        uint32_t *ov0 = reinterpret_cast<uint32_t *>(ord + OL.v0), *ov1 = reinterpret_cast<uint32_t *>(ord + OL.v1);
        uint64_t *gcount = reinterpret_cast<uint64_t *>(ord + OL.gcount);
        if (OL.G > 0)
            hipLaunchKernelGGL(k_order_keys, dim3((unsigned)((OL.G + 255) / 256)), dim3(256), 0, s,
                               proj->ntiles, proj->depth, n, OL.G, ok0, ov0, gcount);
        LEGS_CHECK_LAUNCH(ctx);
        const int gpass = (32 + bits_for(n_views) + 7) / 8;
        if (OL.G > 0) {
            const int32_t r = radix_passes(ctx, sort_scratch_at(ord + OL.sort, OL.G), ok0, ov0, ok1, ov1,
                                           gcount, OL.G, 0, gpass, s);
            if (r != LEGS_OK) return r;
        }
        perm = (gpass % 2 == 0) ? ov0 : ov1;
        nblocks = OL.nbs;
        uint64_t *bcounts = reinterpret_cast<uint64_t *>(ord + OL.bcounts);
        offsets = reinterpret_cast<uint64_t *>(ord + OL.offsets);
        if (nblocks > 0)
            hipLaunchKernelGGL(k_sorted_block_counts, dim3((unsigned)nblocks), dim3(LEGS_PROJ_BLOCK), 0, s,
                               perm, proj->ntiles, OL.G, bcounts);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, bcounts, offsets, nblocks, bins->count);
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
                                       passes, s);
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

    // 2. per-tile counts of the depth-ordered stream (cut at the capacity),
    //    tile ranges and the tile-digit histograms
    const int tbits = bits_for(total_tiles);
    const int np = tbits > 8 ? (tbits + 7) / 8 : 1;
    const int gclear = grid_for(ctx, S.parts * 256 * np, 256, 8);
    hipLaunchKernelGGL(k_sort_clear, dim3(gclear), dim3(256), 0, s, S.status, S.parts, np,
                       S.counters, S.hist, bins->count, bins->capacity);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(ctx, total_tiles, 256, 8)), dim3(256), 0, s,
                       S.tcount, total_tiles, 0u);
    LEGS_CHECK_LAUNCH(ctx);
    if (nblocks > 0)
        hipLaunchKernelGGL(k_tile_corners, dim3((unsigned)nblocks), dim3(256), 0, s, perm,
                           reinterpret_cast<const int4 *>(proj->box), proj->ntiles, offsets, n,
                           OL.G, views, o->tile, bins->capacity, S.tcount);
    LEGS_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(k_tile_rows, dim3(64, (unsigned)n_views), dim3(256), 0, s, S.tcount, views);
    hipLaunchKernelGGL(k_tile_cols, dim3(8, (unsigned)n_views), dim3(256), 0, s, S.tcount, views);
    hipLaunchKernelGGL(k_tile_block_sums, dim3((unsigned)S.tile_blocks), dim3(1024), 0, s, S.tcount,
                       total_tiles, S.tsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, S.tsum, S.toff, S.tile_blocks,
                       S.toff + S.tile_blocks + 1);
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)S.tile_blocks), dim3(1024), 0, s, S.tcount,
                       total_tiles, S.toff, np, bins->ranges, S.hist);
    hipLaunchKernelGGL(k_digit_starts, dim3(np), dim3(256), 0, s, S.hist, S.starts, 0);
    LEGS_CHECK_LAUNCH(ctx);

    // 3. tile passes over 32-bit tile keys: the first generates the instances
    //    from the depth-ordered G-views, the last writes the 64-bit keys; the
    //    32-bit keys ping-pong in the two halves of keys_alt, the ids end in ids
    uint32_t *tk[2] = {reinterpret_cast<uint32_t *>(bins->keys_alt),
                       reinterpret_cast<uint32_t *>(bins->keys_alt) + bins->capacity};
    uint32_t *tv[2] = {bins->ids, bins->ids_alt};
    TileEmit E;
    E.perm = perm;
    E.box = reinterpret_cast<const int4 *>(proj->box);
    E.ntiles = proj->ntiles;
    E.goff = offsets;
    E.nblocks = nblocks;
    E.n = n;
    E.G = OL.G;
    E.views = views;
    E.tile = o->tile;
    TileFinal F;
    F.keys64 = bins->keys;
    F.depth = proj->depth;
    F.n = n;
    F.views = views;
    F.n_views = n_views;
    const int gsort = grid_for(ctx, bins->capacity, LEGS_SORT_PART, 2);
    for (int p = 0; p < np; ++p) {
        // pass p writes buffer (np - 1 - p) % 2, so the last pass writes ids, and
        // reads what the pass before it wrote
        const int wo = (np - 1 - p) % 2, ri = 1 - wo;
        uint64_t *st = S.status + (int64_t)p * S.parts * 256;
        uint32_t *ctr = S.counters + p;
        const bool emit = p == 0, fin = p == np - 1;
        if (emit && fin)
            hipLaunchKernelGGL((k_onesweep<uint32_t, true, true>), dim3(gsort), dim3(LEGS_SORT_THREADS), 0, s,
                               tk[ri], tv[ri], tk[wo], tv[wo], bins->count, bins->capacity, p, S.starts,
                               st, ctr, E, F);
        else if (emit)
            hipLaunchKernelGGL((k_onesweep<uint32_t, true, false>), dim3(gsort), dim3(LEGS_SORT_THREADS), 0, s,
                               tk[ri], tv[ri], tk[wo], tv[wo], bins->count, bins->capacity, p, S.starts,
                               st, ctr, E, F);
        else if (fin)
            hipLaunchKernelGGL((k_onesweep<uint32_t, false, true>), dim3(gsort), dim3(LEGS_SORT_THREADS), 0, s,
                               tk[ri], tv[ri], tk[wo], tv[wo], bins->count, bins->capacity, p, S.starts,
                               st, ctr, E, F);
        else
            hipLaunchKernelGGL((k_onesweep<uint32_t, false, false>), dim3(gsort), dim3(LEGS_SORT_THREADS), 0, s,
                               tk[ri], tv[ri], tk[wo], tv[wo], bins->count, bins->capacity, p, S.starts,
                               st, ctr, E, F);
        LEGS_CHECK_LAUNCH(ctx);
    }
    return LEGS_OK;
}
