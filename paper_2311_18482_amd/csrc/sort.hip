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

// One record per depth-ordered position: everything the tile passes need of
// the G-view there, read once with one coalesced load.
struct GRec {
    uint32_t gid;    // Gaussian index
    uint32_t cnt;    // tiles of its rectangle (0: culled)
    uint32_t base;   // global id of its first tile
    uint32_t rwtx;   // rectangle width | tiles_x of its view << 16
};

// Inputs of the fused emission (first tile pass of the depth-first binning):
// the records of the depth-ordered G-views, the instance offset of every 256
// of them and the first block of each partition.
struct TileEmit {
    const GRec *recs;
    const uint32_t *dbits;
    const uint64_t *goff;      // [nblocks + 1]
    const uint32_t *pstart;    // [partitions]
    int64_t nblocks, G;
};

// Inclusive maximum over lanes 0..l of a wave (DPP row shifts, then the row
// broadcasts of lanes 15 and 31).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x)
{
    uint32_t t;
#define LEGS_DPP_MAX(ctrl, rmask)                                                               \
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, ctrl, rmask, 0xF, false);             \
    x = t > x ? t : x;
    LEGS_DPP_MAX(0x111, 0xF)   // row_shr:1
    LEGS_DPP_MAX(0x112, 0xF)   // row_shr:2
    LEGS_DPP_MAX(0x114, 0xF)   // row_shr:4
    LEGS_DPP_MAX(0x118, 0xF)   // row_shr:8
    LEGS_DPP_MAX(0x142, 0xA)   // row_bcast:15 into rows 1 and 3
    LEGS_DPP_MAX(0x143, 0xC)   // row_bcast:31 into rows 2 and 3
#undef LEGS_DPP_MAX
    return x;
}

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

// LDS of the fused emission.
struct EmitLds {
    uint32_t rbase[256], rwtx[256], rg[256], rd[256];
    uint16_t own[LEGS_SORT_PART];
    uint32_t omax[LEGS_SORT_THREADS / LEGS_WAVE];
    uint64_t gscan[257];
    uint64_t w64[LEGS_SORT_THREADS / LEGS_WAVE];
};

// Generates instances [base, base + nvalid) of the depth-ordered stream into
// LDS slots 0 .. nvalid - 1 (tile key, Gaussian id, depth bits): instance e is
// tile e - start of its G-view's rectangle, row-major. Each G-view marks the
// first slot it fills and a running maximum over the slots gives every slot
// its owner. Called by the whole workgroup.
template <typename K, bool DEP>
__device__ __forceinline__ void emit_partition(const TileEmit &E, int64_t part, int64_t base, int nvalid,
                                               K *s_keys, uint32_t *s_vals, uint32_t *s_dep, EmitLds &M)
{
    constexpr int T = LEGS_SORT_THREADS;
    constexpr int NW = T / LEGS_WAVE;
    constexpr int SPW = LEGS_SORT_PART / NW;   // partition slots per wave
    const int tid = threadIdx.x, lane = legs_lane(), wave = tid / LEGS_WAVE;
    for (int64_t b = E.pstart[part]; b < E.nblocks; ++b) {
        const uint64_t ob = E.goff[b];
        if (ob >= (uint64_t)(base + nvalid)) break;
        const int64_t pos = b * 256 + tid;
        uint32_t c = 0;
        if (tid < 256 && pos < E.G) {
            const GRec r = E.recs[pos];
            c = r.cnt;
            M.rbase[tid] = r.base;
            M.rwtx[tid] = r.rwtx;
            M.rg[tid] = r.gid;
            M.rd[tid] = c ? E.dbits[pos] : 0u;
        }
        block_scan_256<T>(c, M.gscan, M.w64);
        const uint64_t tot = M.gscan[256];
        const uint64_t lo = (uint64_t)base > ob ? (uint64_t)base - ob : 0;
        const uint64_t hi = ((uint64_t)(base + nvalid) - ob) < tot ? (uint64_t)(base + nvalid) - ob : tot;
        const int e_lo = (int)(ob + lo - (uint64_t)base), e_hi = (int)(ob + hi - (uint64_t)base);
        // clear the slots of this block, mark each G-view's first slot; wave w
        // owns slots [w SPW, (w + 1) SPW), lane-contiguous in chunks of 64
#pragma unroll
        for (int q = 0; q < SPW / LEGS_WAVE; ++q) {
            const int e = wave * SPW + q * LEGS_WAVE + lane;
            if (e >= e_lo && e < e_hi) M.own[e] = 0;
        }
        __syncthreads();
        if (tid < 256 && c) {
            const uint64_t st = M.gscan[tid];
            const uint64_t first = st > lo ? st : lo;
            if (first < hi && first < st + c) M.own[(int)(ob + first - (uint64_t)base)] = (uint16_t)(tid + 1);
        }
        __syncthreads();
        // owner of each slot: running maximum of the marks (per-wave maxima
        // first, then a DPP max-scan per chunk carried across chunks)
        uint32_t wm = 0;
#pragma unroll
        for (int q = 0; q < SPW / LEGS_WAVE; ++q) {
            const int e = wave * SPW + q * LEGS_WAVE + lane;
            const uint32_t mk = (e >= e_lo && e < e_hi) ? (uint32_t)M.own[e] : 0u;
            wm = mk > wm ? mk : wm;
        }
        wm = wave_incl_max(wm);
        if (lane == LEGS_WAVE - 1) M.omax[wave] = wm;
        __syncthreads();
        uint32_t carry = 0;
        for (int w = 0; w < wave; ++w) carry = M.omax[w] > carry ? M.omax[w] : carry;
#pragma unroll
        for (int q = 0; q < SPW / LEGS_WAVE; ++q) {
            const int e = wave * SPW + q * LEGS_WAVE + lane;
            const bool in = e >= e_lo && e < e_hi;
            uint32_t own = wave_incl_max(in ? (uint32_t)M.own[e] : 0u);
            own = own > carry ? own : carry;
            carry = (uint32_t)__builtin_amdgcn_readlane((int)own, LEGS_WAVE - 1);
            if (in) {
                const int o = (int)own - 1;
                const uint32_t local = (uint32_t)((uint64_t)base + (uint64_t)e - ob - M.gscan[o]);
                const uint32_t rwtx = M.rwtx[o], rw = rwtx & 0xffffu, tx = rwtx >> 16;
                // local / rw through a float reciprocal (local < 2^24, rw < 2^16:
                // the estimate is off by at most a few units, fixed below)
                uint32_t qq = (uint32_t)((float)local * __builtin_amdgcn_rcpf((float)rw));
                int32_t rr = (int32_t)(local - qq * rw);
                while (rr < 0) { --qq; rr += (int32_t)rw; }
                while (rr >= (int32_t)rw) { ++qq; rr -= (int32_t)rw; }
                s_keys[e] = (K)(M.rbase[o] + qq * tx + (uint32_t)rr);
                s_vals[e] = M.rg[o];
                if constexpr (DEP) s_dep[e] = M.rd[o];
            }
        }
        __syncthreads();
    }
}

// One onesweep pass over digit `pass` (bits 8 pass .. 8 pass + 7) of keys K
// with 32-bit values, and with DEP a second 32-bit value (the depth bits)
// carried along. EMIT: the partition's (tile, id, depth) triples are
// generated from the depth-ordered G-view records instead of read (instance
// e is tile e - start of its G-view's rectangle, row-major): each G-view
// marks the first partition slot it fills, and a running maximum over the
// slots gives every slot its owner. FINAL: the keys are written as the 64-bit
// (tile << 32) | depth keys of the tile lists.
template <typename K, bool DEP, bool EMIT, bool FINAL, bool SEG>
__global__ void __launch_bounds__(LEGS_SORT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
k_onesweep(const K *__restrict__ kin, const uint32_t *__restrict__ vin,
           const uint32_t *__restrict__ din, K *__restrict__ kout, uint32_t *__restrict__ vout,
           uint32_t *__restrict__ dout, uint64_t *__restrict__ keys64,
           const uint64_t *__restrict__ count, int64_t capacity, int pass, int shift, int rb,
           const uint32_t *__restrict__ digit_starts, uint64_t *__restrict__ status,
           uint32_t *__restrict__ counter, TileEmit E, const uint32_t *__restrict__ seg_off)
{
    constexpr int T = LEGS_SORT_THREADS;
    constexpr int NW = T / LEGS_WAVE;
    constexpr int ITEMS = LEGS_SORT_ITEMS;
    constexpr int PART = LEGS_SORT_PART;
    static_assert(T >= 256 && T % 256 == 0, "one thread per digit");
    __shared__ K s_keys[PART];
    __shared__ uint32_t s_vals[PART];
    __shared__ uint32_t s_dep[DEP ? PART : 1];
    __shared__ uint32_t s_wh[NW][256];      // per-wave digit counts, then wave offsets
    __shared__ uint32_t s_lstart[256];      // block-local start of each digit
    __shared__ uint64_t s_gstart[257];      // global position of LDS slot 0 of each digit;
                                            // with EMIT first the G-view scan of a block
    __shared__ uint32_t s_tmp[NW];
    __shared__ uint64_t s_w64[NW];
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

        if constexpr (EMIT) {
            __shared__ EmitLds s_emit;
            emit_partition<K, DEP>(E, part, base, nvalid, s_keys, s_vals, s_dep, s_emit);
        }

        K key[ITEMS];
        uint32_t val[ITEMS], dep[DEP ? ITEMS : 1];
        uint32_t rank[ITEMS];
        // wave-striped: item i of lane l of wave w is partition element w*64*ITEMS + i*64 + l
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int e = wave * LEGS_WAVE * ITEMS + i * LEGS_WAVE + lane;
            if (e < nvalid) {
                if constexpr (EMIT) {
                    key[i] = s_keys[e];
                    val[i] = s_vals[e];
                    if constexpr (DEP) dep[i] = s_dep[e];
                } else {
                    key[i] = kin[base + e];
                    val[i] = vin[base + e];
                    if constexpr (DEP) dep[i] = din[base + e];
                }
            } else {
                key[i] = (K)~(K)0;
                val[i] = 0;
                if constexpr (DEP) dep[i] = 0;
            }
        }
        if constexpr (EMIT) __syncthreads();   // the LDS arrays are reused by the scatter below
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
                s_vals[pos] = val[i];
                if constexpr (DEP) s_dep[pos] = dep[i];
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
                constexpr int LB = 16;
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
            s_gstart[d] = (uint64_t)digit_starts[pass * 256 + d] + excl - (uint64_t)lstart;
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
                    if constexpr (FINAL) {
                        keys64[gpos] = ((uint64_t)kk << 32) | s_dep[k];
                        vout[gpos] = s_vals[k];
                    } else {
                        kout[gpos] = kk;
                        vout[gpos] = s_vals[k];
                        if constexpr (DEP) dout[gpos] = s_dep[k];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Digit counts of pass `pass` over the partitions of segment blockIdx.x (the
// same segments as the segment passes: per = ceil(partitions / gridDim.x)).
__global__ void __launch_bounds__(LEGS_SORT_THREADS)
k_tile_upsweep(const uint32_t *__restrict__ kin, const uint64_t *__restrict__ count, int64_t capacity,
               int shift, int rb, uint32_t *__restrict__ seg_hist)
{
    constexpr int T = LEGS_SORT_THREADS, PART = LEGS_SORT_PART, ITEMS = LEGS_SORT_ITEMS;
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
        for (int q = 0; q < ITEMS; ++q)
            if (tid + q * T < nvalid) atomicAdd(&s_hist[(k[q] >> shift) & dmask], 1u);
    }
    __syncthreads();
    if (tid < 256) seg_hist[(int64_t)blockIdx.x * 256 + tid] = s_hist[tid];
}

// Start of every digit run of every segment: the digit's global start plus the
// counts of the segments before. One workgroup per digit, one thread per
// segment (nseg <= LEGS_SEG_MAX).
__global__ void __launch_bounds__(LEGS_SEG_MAX)
k_seg_scan(const uint32_t *__restrict__ seg_hist, int nseg, const uint32_t *__restrict__ digit_starts,
           int pass, uint32_t *__restrict__ seg_off)
{
    __shared__ uint32_t s_w[LEGS_SEG_MAX / LEGS_WAVE];
    const int d = blockIdx.x, sg = threadIdx.x;
    const int lane = legs_lane(), wave = sg / LEGS_WAVE;
    const uint32_t x = sg < nseg ? seg_hist[(int64_t)sg * 256 + d] : 0u;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    if (lane == LEGS_WAVE - 1) s_w[wave] = incl;
    __syncthreads();
    uint32_t pre = digit_starts[pass * 256 + d];
    for (int w = 0; w < wave; ++w) pre += s_w[w];
    if (sg < nseg) seg_off[(int64_t)sg * 256 + d] = pre + incl - x;
}

// Counts of the low rb bits of the tile ids in segment blockIdx.x of the
// depth-ordered stream (the first tile pass), from the G-view records without
// generating the instances: every row of a rectangle covers consecutive tile
// ids, i.e. a cyclic range of digits, added to a difference array (full turns
// of 2^rb to every digit at once).
__global__ void __launch_bounds__(256)
k_tile_upsweep_emit(const uint64_t *__restrict__ count, int64_t capacity, TileEmit E, int rb,
                    uint32_t *__restrict__ seg_hist)
{
    const uint32_t nd = 1u << rb;   // the first pass sorts the low rb bits of the tile id
    constexpr int PART = LEGS_SORT_PART;
    __shared__ uint32_t s_d[257];
    __shared__ uint32_t s_all;
    __shared__ uint64_t s_start[257];
    __shared__ uint64_t s_w[4];
    const int tid = threadIdx.x;
    for (int i = tid; i < 257; i += 256) s_d[i] = 0;
    if (tid == 0) s_all = 0;
    const uint64_t cnt = *count;
    const int64_t m = (int64_t)(cnt < (uint64_t)capacity ? cnt : (uint64_t)capacity);
    const int64_t parts = (m + PART - 1) / PART;
    const int64_t per = (parts + gridDim.x - 1) / gridDim.x;
    const int64_t p0 = (int64_t)blockIdx.x * per;
    __syncthreads();
    if (p0 < parts) {
        const uint64_t s0 = (uint64_t)p0 * PART;
        const uint64_t s1 = (uint64_t)((p0 + per) * PART < m ? (p0 + per) * PART : m);
        for (int64_t b = E.pstart[p0]; b < E.nblocks; ++b) {
            const uint64_t ob = E.goff[b];
            if (ob >= s1) break;
            const int64_t pos = b * 256 + tid;
            const GRec r = pos < E.G ? E.recs[pos] : GRec{0u, 0u, 0u, 0u};
            block_scan_256<256>(r.cnt, s_start, s_w);
            const uint64_t st = ob + s_start[tid];
            const uint64_t u0g = st > s0 ? st : s0, u1g = st + r.cnt < s1 ? st + r.cnt : s1;
            if (r.cnt && u0g < u1g) {
                const uint32_t rw = r.rwtx & 0xffffu, tx = r.rwtx >> 16;
                const uint32_t u0 = (uint32_t)(u0g - st), u1 = (uint32_t)(u1g - st);   // [u0, u1) of the rectangle
                for (uint32_t row = u0 / rw; row * rw < u1; ++row) {
                    const uint32_t c0 = row * rw < u0 ? u0 - row * rw : 0u;
                    const uint32_t c1 = (row + 1) * rw < u1 ? rw : u1 - row * rw;   // columns [c0, c1)
                    const uint32_t a = (r.base + row * tx + c0) & (nd - 1u), len = c1 - c0;
                    if (len >> rb) atomicAdd(&s_all, len >> rb);
                    const uint32_t rem = len & (nd - 1u);
                    if (rem) {
                        atomicAdd(&s_d[a], 1u);
                        if (a + rem <= nd) {
                            atomicAdd(&s_d[a + rem], 0xffffffffu);
                        } else {
                            atomicAdd(&s_d[nd], 0xffffffffu);
                            atomicAdd(&s_d[0], 1u);
                            atomicAdd(&s_d[a + rem - nd], 0xffffffffu);
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    // inclusive prefix of the difference array over the 256 bytes
    const int lane = legs_lane(), wave = tid / LEGS_WAVE;
    uint32_t incl = s_d[tid];
#pragma unroll
    for (int off = 1; off < LEGS_WAVE; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, LEGS_WAVE);
        if (lane >= off) incl += y;
    }
    __shared__ uint32_t s_t[4];
    if (lane == LEGS_WAVE - 1) s_t[wave] = incl;
    __syncthreads();
    for (int w = 0; w < wave; ++w) incl += s_t[w];
    seg_hist[(int64_t)blockIdx.x * 256 + tid] = (uint32_t)tid < nd ? incl + s_all : 0u;
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

// Records, depth bits and per-view position ranges of the depth-ordered
// G-views, and the instance count of each block of 256 positions.
__global__ void __launch_bounds__(LEGS_PROJ_BLOCK)
k_sorted_records(const uint32_t *__restrict__ perm, const uint64_t *__restrict__ okeys,
                 const int4 *__restrict__ box, const float *__restrict__ depth,
                 const uint32_t *__restrict__ ntiles, int64_t n, int64_t G,
                 const legs_view *__restrict__ views, int tile, GRec *__restrict__ recs,
                 uint32_t *__restrict__ dbits, uint64_t *__restrict__ vrange,
                 uint64_t *__restrict__ block_counts)
{
    const int64_t pos = (int64_t)blockIdx.x * LEGS_PROJ_BLOCK + threadIdx.x;
    uint64_t c = 0;
    if (pos < G) {
        const int64_t gv = perm[pos];
        c = ntiles[gv];
        GRec r = {0u, 0u, 0u, 0u};
        if (c) {
            const int64_t v = gv / n;
            const int4 bx = box[gv];
            const legs_view &vw = views[v];
            const int tx0 = bx.x / tile, ty0 = bx.z / tile;
            r.gid = (uint32_t)(gv - v * n);
            r.cnt = (uint32_t)c;
            r.base = (uint32_t)(vw.tile_offset + (int64_t)ty0 * vw.tiles_x + tx0);
            r.rwtx = (uint32_t)(bx.y / tile - tx0 + 1) | ((uint32_t)vw.tiles_x << 16);
            dbits[pos] = __float_as_uint(depth[gv]);
            // first and last position of each view (visible G-views sort by view)
            const uint64_t kv = okeys[pos] >> 32;
            if (pos == 0 || (okeys[pos - 1] >> 32) != kv) vrange[2 * kv] = (uint64_t)pos;
            if (pos == G - 1 || (okeys[pos + 1] >> 32) != kv) vrange[2 * kv + 1] = (uint64_t)pos + 1;
        }
        recs[pos] = r;
    }
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

// First block of 256 positions of every partition of the instance stream:
// partition p starts in block b when goff[b] <= p * PART < goff[b + 1].
__global__ void __launch_bounds__(256)
k_part_blocks(const uint64_t *__restrict__ goff, int64_t nblocks, int64_t parts_cap,
              uint32_t *__restrict__ pstart)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= nblocks) return;
    const int64_t plo = (int64_t)((goff[b] + LEGS_SORT_PART - 1) / LEGS_SORT_PART);
    int64_t phi = (int64_t)((goff[b + 1] + LEGS_SORT_PART - 1) / LEGS_SORT_PART);
    if (phi > parts_cap) phi = parts_cap;
    for (int64_t p = plo; p < phi; ++p) pstart[p] = (uint32_t)b;
}

// ---- per-tile counts of the depth-ordered instance stream ----------------------

// The first `capacity` instances of the depth-ordered stream are counted per
// tile on a 2D difference array (the tile grid of each view): +1 / -1 at the
// corners of each G-view's tile rectangle, then prefix sums along the rows and
// the columns. A G-view cut by the capacity contributes its first tiles in
// row-major order (full rows plus one partial row). The counts give the
// tile ranges and the digit histograms of the tile passes without reading
// the instances.
// +1 / -1 at the corners of a tile rectangle (view-local tile coordinates).
__device__ __forceinline__ void diff_rect(uint32_t *g, int W, int H, int x0, int x1, int y0, int y1)
{
    atomicAdd(g + y0 * W + x0, 1u);
    if (x1 + 1 < W) atomicAdd(g + y0 * W + x1 + 1, 0xffffffffu);
    if (y1 + 1 < H) atomicAdd(g + (y1 + 1) * W + x0, 0xffffffffu);
    if (x1 + 1 < W && y1 + 1 < H) atomicAdd(g + (y1 + 1) * W + x1 + 1, 1u);
}

constexpr int TILE_LDS_CELLS = 16384;   // views with at most this many tiles count in LDS

// Workgroup (c, v) adds the rectangles of view v's G-views in position blocks
// c, c + gridDim.x, ... into an LDS copy of the view's tile grid and stores it
// in partial[c] (views with more tiles than fit add straight into the global
// grid with atomics); k_tile_merge then sums the partial grids. Hot corner
// cells cost LDS atomics instead of global ones.
__global__ void __launch_bounds__(256)
k_tile_corners(const GRec *__restrict__ recs, const uint64_t *__restrict__ goff,
               const uint64_t *__restrict__ vrange, int64_t G,
               const legs_view *__restrict__ views, int64_t capacity, int64_t total_tiles,
               uint32_t *__restrict__ diff, uint32_t *__restrict__ partial)
{
    __shared__ uint32_t s_grid[TILE_LDS_CELLS];
    __shared__ uint64_t s_start[257];
    __shared__ uint64_t s_w[4];
    const int v = blockIdx.y;
    const legs_view vw = views[v];
    const int W = vw.tiles_x, H = vw.tiles_y;
    const int ncell = W * H;
    const bool lds = ncell <= TILE_LDS_CELLS;
    uint32_t *g = lds ? s_grid : diff + vw.tile_offset;
    if (lds)
        for (int i = threadIdx.x; i < ncell; i += 256) s_grid[i] = 0u;
    const int64_t p0 = (int64_t)vrange[2 * v], p1 = (int64_t)vrange[2 * v + 1];
    __syncthreads();
    if (p1 > p0) {
        for (int64_t b = p0 / 256 + blockIdx.x; b <= (p1 - 1) / 256; b += gridDim.x) {
            const int64_t pos = b * 256 + threadIdx.x;
            const GRec r = pos < G ? recs[pos] : GRec{0u, 0u, 0u, 0u};
            block_scan_256<256>(r.cnt, s_start, s_w);
            const uint64_t off = goff[b] + s_start[threadIdx.x];
            if (pos >= p0 && pos < p1 && r.cnt && off < (uint64_t)capacity) {
                const uint64_t keep = (uint64_t)capacity - off < r.cnt ? (uint64_t)capacity - off : r.cnt;
                const int rw = (int)(r.rwtx & 0xffffu);
                const int local = (int)((int64_t)r.base - vw.tile_offset);
                const int x0 = local % W, y0 = local / W;
                const int rows = (int)(r.cnt / (uint32_t)rw);
                if (keep == r.cnt) {
                    diff_rect(g, W, H, x0, x0 + rw - 1, y0, y0 + rows - 1);
                } else {
                    const int full = (int)(keep / (uint64_t)rw), rem = (int)(keep % (uint64_t)rw);
                    if (full > 0) diff_rect(g, W, H, x0, x0 + rw - 1, y0, y0 + full - 1);
                    if (rem > 0) diff_rect(g, W, H, x0, x0 + rem - 1, y0 + full, y0 + full);
                }
            }
            __syncthreads();
        }
    }
    if (lds) {
        __syncthreads();
        uint32_t *out = partial + (int64_t)blockIdx.x * total_tiles + vw.tile_offset;
        for (int i = threadIdx.x; i < ncell; i += 256) out[i] = s_grid[i];
    }
}

// Sum of the partial grids of views counted in LDS (the others already hold
// their counts in diff).
__global__ void __launch_bounds__(256)
k_tile_merge(const uint32_t *__restrict__ partial, int nch, int64_t total_tiles,
             const legs_view *__restrict__ views, int n_views, uint32_t *__restrict__ diff)
{
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total_tiles; t += (int64_t)gridDim.x * 256) {
        const legs_view &vw = views[legs_view_of_tile(views, n_views, t)];
        if (vw.tiles_x * vw.tiles_y > TILE_LDS_CELLS) continue;
        uint32_t acc = 0;
#pragma unroll 8
        for (int c = 0; c < nch; ++c) acc += partial[(int64_t)c * total_tiles + t];
        diff[t] = acc;
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
// histograms of the tile passes (pass p's digit: the next (widths >> 4p) & 15
// bits of the tile id).
__global__ void __launch_bounds__(1024)
k_tile_ranges(const uint32_t *__restrict__ counts, int64_t total_tiles,
              const uint64_t *__restrict__ boff, int npass, uint32_t widths, uint32_t *__restrict__ ranges,
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
        if (x) {
            int sh = 0;
            for (int p = 0; p < npass; ++p) {
                const int w = (int)((widths >> (4 * p)) & 15u);
                atomicAdd(&s_h[p][(uint32_t)(t >> sh) & ((1u << w) - 1u)], (uint32_t)x);
                sh += w;
            }
        }
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
    L.pstart_off = (L.toff_off + 8 * (L.tile_blocks + 1) + 8 + 255) & ~(int64_t)255;
    const int64_t np_ = total_tiles > 0 ? L.parts : 0;    // the G-view sort needs none of these
    L.dep_off = (L.pstart_off + 4 * np_ + 255) & ~(int64_t)255;
    L.part_off = (L.dep_off + (total_tiles > 0 ? 8 * capacity : 0) + 255) & ~(int64_t)255;
    L.seg_off = (L.part_off + 4 * (int64_t)LEGS_TILE_CHUNKS * total_tiles + 255) & ~(int64_t)255;
    L.total = L.seg_off + (total_tiles > 0 ? 2 * 4 * (int64_t)LEGS_SEG_MAX * 256 : 0);
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
    uint32_t *pstart, *dep, *partial, *seg_hist, *seg_off;
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
    S.pstart = reinterpret_cast<uint32_t *>(b + L.pstart_off);
    S.dep = reinterpret_cast<uint32_t *>(b + L.dep_off);
    S.partial = reinterpret_cast<uint32_t *>(b + L.part_off);
    S.seg_hist = reinterpret_cast<uint32_t *>(b + L.seg_off);
    S.seg_off = S.seg_hist + (int64_t)LEGS_SEG_MAX * 256;
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
        hipLaunchKernelGGL((k_onesweep<uint64_t, false, false, false, false>), dim3(gsort),
                           dim3(LEGS_SORT_THREADS), 0, s, ka, va, nullptr, kb, vb, nullptr, nullptr, count,
                           capacity, p, 8 * p, 8, S.starts, S.status + (int64_t)(p - first) * S.parts * 256,
                           S.counters + (p - first), TileEmit{}, nullptr);
        LEGS_CHECK_LAUNCH(ctx);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    return LEGS_OK;
}

struct OrderLayout {
    int64_t G, nbs;
    int64_t k0, k1, v0, v1, bcounts, offsets, gcount, recs, dbits, vrange, sort, total;
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
    L.recs = o; o = align256(o + 16 * L.G);
    L.dbits = o; o = align256(o + 4 * L.G);
    L.vrange = o; o = align256(o + 16 * (int64_t)n_views);
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
        uint64_t *vrange = reinterpret_cast<uint64_t *>(ord + OL.vrange);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, reinterpret_cast<uint32_t *>(vrange),
                           (int64_t)4 * n_views, 0u);
        if (nblocks > 0)
            hipLaunchKernelGGL(k_sorted_records, dim3((unsigned)nblocks), dim3(LEGS_PROJ_BLOCK), 0, s,
                               perm, (gpass % 2 == 0) ? ok0 : ok1,
                               reinterpret_cast<const int4 *>(proj->box), proj->depth, proj->ntiles,
                               n, OL.G, views, o->tile, reinterpret_cast<GRec *>(ord + OL.recs),
                               reinterpret_cast<uint32_t *>(ord + OL.dbits), vrange, bcounts);
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
    const GRec *recs = reinterpret_cast<const GRec *>(ord + OL.recs);
    const uint64_t *vrange = reinterpret_cast<const uint64_t *>(ord + OL.vrange);
    // tile-id bits split as evenly as possible over ceil(bits / 8) passes (13 bits:
    // 7 + 6), so digit runs stay long and the match needs fewer ballots
    const int tbits = bits_for(total_tiles) > 0 ? bits_for(total_tiles) : 1;
    const int np = (tbits + 7) / 8;
    int pw[4] = {0, 0, 0, 0}, psh[4] = {0, 0, 0, 0};
    uint32_t widths = 0;
    for (int p = 0, sh = 0; p < np; ++p) {
        pw[p] = tbits / np + (p < tbits % np ? 1 : 0);
        psh[p] = sh;
        sh += pw[p];
        widths |= (uint32_t)pw[p] << (4 * p);
    }
    hipLaunchKernelGGL(k_sort_clear, dim3(1), dim3(256), 0, s, S.status, S.parts, 0, S.counters,
                       S.hist, bins->count, bins->capacity);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(ctx, total_tiles, 256, 8)), dim3(256), 0, s,
                       S.tcount, total_tiles, 0u);
    LEGS_CHECK_LAUNCH(ctx);
    // enough workgroups per view to spread the G-views, at most LEGS_TILE_CHUNKS
    int nch = (int)(((OL.G / (n_views > 0 ? n_views : 1)) + 8191) / 8192);
    nch = nch < 1 ? 1 : (nch > LEGS_TILE_CHUNKS ? LEGS_TILE_CHUNKS : nch);
    hipLaunchKernelGGL(k_tile_corners, dim3((unsigned)nch, (unsigned)n_views), dim3(256), 0, s, recs,
                       offsets, vrange, OL.G, views, bins->capacity, total_tiles, S.tcount, S.partial);
    hipLaunchKernelGGL(k_tile_merge, dim3(grid_for(ctx, total_tiles, 256, 8)), dim3(256), 0, s,
                       S.partial, nch, total_tiles, views, n_views, S.tcount);
    hipLaunchKernelGGL(k_tile_rows, dim3(64, (unsigned)n_views), dim3(256), 0, s, S.tcount, views);
    hipLaunchKernelGGL(k_tile_cols, dim3(8, (unsigned)n_views), dim3(256), 0, s, S.tcount, views);
    hipLaunchKernelGGL(k_tile_block_sums, dim3((unsigned)S.tile_blocks), dim3(1024), 0, s, S.tcount,
                       total_tiles, S.tsum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, S.tsum, S.toff, S.tile_blocks,
                       S.toff + S.tile_blocks + 1);
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)S.tile_blocks), dim3(1024), 0, s, S.tcount,
                       total_tiles, S.toff, np, widths, bins->ranges, S.hist);
    hipLaunchKernelGGL(k_digit_starts, dim3(np), dim3(256), 0, s, S.hist, S.starts, 0);
    if (nblocks > 0)
        hipLaunchKernelGGL(k_part_blocks, dim3((unsigned)((nblocks + 255) / 256)), dim3(256), 0, s,
                           offsets, nblocks, S.parts, S.pstart);
    LEGS_CHECK_LAUNCH(ctx);

    // 3. tile passes over 32-bit tile keys carrying (id, depth bits): the first
    //    generates the instances from the depth-ordered G-view records, the last
    //    writes the 64-bit keys and the ids. The 32-bit keys ping-pong in the two
    //    halves of keys_alt, the ids between ids_alt and ids, the depth bits in
    //    the sort scratch.
    uint32_t *tk[2] = {reinterpret_cast<uint32_t *>(bins->keys_alt),
                       reinterpret_cast<uint32_t *>(bins->keys_alt) + bins->capacity};
    uint32_t *tv[2] = {bins->ids, bins->ids_alt};
    uint32_t *td[2] = {S.dep, S.dep + bins->capacity};
    TileEmit E;
    E.recs = recs;
    E.dbits = reinterpret_cast<const uint32_t *>(ord + OL.dbits);
    E.goff = offsets;
    E.pstart = S.pstart;
    E.nblocks = nblocks;
    E.G = OL.G;
    // every tile pass: digit counts per segment of partitions, their scan, then
    // the pass itself with each workgroup walking its own segment in order
    const int nseg = (int)(ctx->num_cus * 2 < LEGS_SEG_MAX ? ctx->num_cus * 2 : LEGS_SEG_MAX);
    for (int p = 0; p < np; ++p) {
        // pass p writes buffer (np - 1 - p) % 2 (the last one: ids) and reads
        // what the pass before it wrote
        const int wo = (np - 1 - p) % 2, ri = 1 - wo;
        const bool emit = p == 0, fin = p == np - 1;
        if (emit)
            hipLaunchKernelGGL(k_tile_upsweep_emit, dim3(nseg), dim3(256), 0, s, bins->count, bins->capacity,
                               E, pw[p], S.seg_hist);
        else
            hipLaunchKernelGGL(k_tile_upsweep, dim3(nseg), dim3(LEGS_SORT_THREADS), 0, s, tk[ri],
                               bins->count, bins->capacity, psh[p], pw[p], S.seg_hist);
        hipLaunchKernelGGL(k_seg_scan, dim3(256), dim3(LEGS_SEG_MAX), 0, s, S.seg_hist, nseg, S.starts, p,
                           S.seg_off);
#define LEGS_TILE_PASS(EM, FI)                                                                      \
        hipLaunchKernelGGL((k_onesweep<uint32_t, true, EM, FI, true>), dim3(nseg), dim3(LEGS_SORT_THREADS), \
                           0, s, tk[ri], tv[ri], td[ri], tk[wo], tv[wo], td[wo], bins->keys, bins->count, \
                           bins->capacity, p, psh[p], pw[p], S.starts, nullptr, nullptr, E, S.seg_off)
        if (emit && fin) LEGS_TILE_PASS(true, true);
        else if (emit) LEGS_TILE_PASS(true, false);
        else if (fin) LEGS_TILE_PASS(false, true);
        else LEGS_TILE_PASS(false, false);
#undef LEGS_TILE_PASS
        LEGS_CHECK_LAUNCH(ctx);
    }
    return LEGS_OK;
}
