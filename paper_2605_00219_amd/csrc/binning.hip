// Binning and sorting: exclusive scan of tiles touched, 32-bit (tile, depth)
// key emission, stable LSD radix sort of each view's segment (4 passes of 8
// bits) carrying the Gaussian id, and per-tile [start, end) ranges.  The
// depth part of each key comes precomputed from the projection record.
//
// The sort runs over all views at once: each view's segment is cut into
// chunks of kChunk keys that never straddle two views.  One histogram pass
// gives every view's digit totals for all four passes; each pass is then a
// single kernel in which a chunk's destinations are the digit's start plus
// the counts of the view's earlier chunks, found by a decoupled look-back.
// Grids are sized from the capacity (an upper bound known on the host); the
// actual counts are read on the device, so no step needs a host
// synchronisation.
#include "cull_math.h"
#include "gs_internal.h"

namespace gs {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanBlock = kScanThreads * kScanItems;  // 2048 elements per block
constexpr int kSortThreads = 256;
constexpr int kSortItems = 24;
constexpr int kChunk = kSortThreads * kSortItems;      // 6144 keys per radix chunk
constexpr int kDepthItems = 8;                          // the depth sort of (view, Gaussian)s:
constexpr int kDepthChunk = kSortThreads * kDepthItems; // 2048-key chunks
constexpr int64_t kDepthFirstRatio = 12;                // capacity / (views x n) to sort by depth first
constexpr int kDepthSplit = 16;                          // key bits sorted per Gaussian in the depth order
constexpr int kDigits = 256;
constexpr int kPasses = 4;
constexpr int kHistBlocks = 2048;                       // workgroups of the histogram pass
constexpr int kGroup = 16;                              // chunks per look-back group
// single-pass tile scatter (depth order first, every view with at most
// kTsBins tiles): chunks of kTsChunk keys in depth order
constexpr int kTsThreads = 256;
// 10240 keys: the 4.9M keys of a 300k-Gaussian 720p view make 475 chunks,
// one round of the 512 workgroups two per CU hold (8192 left a second round
// of 82 and took 27 us longer)
constexpr int kTsItems = 40;
constexpr int kTsChunk = kTsThreads * kTsItems;
constexpr int kTsBins = 4096;                            // tiles per view (12 bits)
static_assert(kSortThreads == kDigits, "one thread per digit in the scan and look-back");

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

// Sizes of the sort's device words for n_views segments and max_chunks chunks.
static inline int64_t max_groups_for(int64_t max_chunks, int n_views) {
    return max_chunks / kGroup + n_views + 1;
}

static inline size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

static size_t sort_words_bytes(int n_views, int64_t mc) {
    const int64_t mg = max_groups_for(mc, n_views);
    const size_t nd = (size_t)n_views * kPasses * kDigits;
    return align_up(4 * nd) + align_up(8 * (size_t)(kPasses * mc * kDigits)) * 2 +
           align_up(8 * (size_t)(kPasses * mg * kDigits)) + align_up(4 * (size_t)(kPasses * mg));
}

struct Workspace {
    uint32_t* row_count;   // tile rows per (view, Gaussian)
    uint32_t* keys_tmp;
    uint32_t* vals_tmp;
    uint64_t* block_sums;  // scan partials
    uint32_t* table;       // 4 * (GS_MAX_VIEWS + 1)
    uint32_t* sort_words;  // the sort's totals and look-back words (carve_sort)
    int64_t max_chunks;
    // depth order of the (view, Gaussian)s
    uint32_t *dkey, *dval, *dkey_tmp, *dval_tmp;
    uint32_t* dpos;        // per (view, Gaussian): its first position in depth order
    uint64_t* dblock_sums; // scan partials of the depth-order scan (runs beside the others)
    uint32_t* dtable;      // segments of the depth sort
    uint32_t* dsort_words;
    int64_t max_dchunks;
    // single-pass tile scatter
    uint32_t* tstable;     // 4 * (GS_MAX_VIEWS + 1): per view chunk base, chunks, matrix base, tiles
    uint32_t* tsm;         // per view, tiles x chunks key counts, scanned in place (+1 word)
    uint64_t* ts_sums;     // scan partials of tsm
    int64_t max_ts_chunks;
    int64_t ts_len;        // words of tsm scanned (an upper bound of the used length)
};

static int max_view_tiles(const gs_layout& L) {
    int mt = 0;
    for (int v = 0; v < L.n_views; ++v) mt = std::max(mt, L.tile_base[v + 1] - L.tile_base[v]);
    return mt;
}

static int64_t max_chunks_for(int64_t capacity, int n_views) {
    return (capacity + kChunk - 1) / kChunk + n_views;
}

static size_t carve(int64_t n, const gs_layout& L, int64_t capacity, char* base, Workspace* w) {
    const int64_t mc = max_chunks_for(capacity, L.n_views);
    const int64_t sb = ((int64_t)L.n_views * n + kScanBlock - 1) / kScanBlock + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    Workspace tmp;
    tmp.row_count = (uint32_t*)take(sizeof(uint32_t) * (size_t)std::max<int64_t>((int64_t)L.n_views * n, 1));
    tmp.keys_tmp = (uint32_t*)take(sizeof(uint32_t) * (size_t)std::max<int64_t>(capacity, 1));
    tmp.vals_tmp = (uint32_t*)take(sizeof(uint32_t) * (size_t)std::max<int64_t>(capacity, 1));
    tmp.block_sums = (uint64_t*)take(sizeof(uint64_t) * (size_t)(sb + 1));
    tmp.table = (uint32_t*)take(sizeof(uint32_t) * 4 * (GS_MAX_VIEWS + 1));
    tmp.sort_words = (uint32_t*)take(sort_words_bytes(L.n_views, mc));
    tmp.max_chunks = mc;
    const int64_t m = std::max<int64_t>((int64_t)L.n_views * n, 1);
    const int64_t mcd = (m + kDepthChunk - 1) / kDepthChunk + L.n_views;
    tmp.dkey = (uint32_t*)take(sizeof(uint32_t) * (size_t)m);
    tmp.dval = (uint32_t*)take(sizeof(uint32_t) * (size_t)m);
    tmp.dkey_tmp = (uint32_t*)take(sizeof(uint32_t) * (size_t)m);
    tmp.dval_tmp = (uint32_t*)take(sizeof(uint32_t) * (size_t)m);
    tmp.dpos = (uint32_t*)take(sizeof(uint32_t) * (size_t)m);
    tmp.dblock_sums = (uint64_t*)take(sizeof(uint64_t) * (size_t)(sb + 1));
    tmp.dtable = (uint32_t*)take(sizeof(uint32_t) * 4 * (GS_MAX_VIEWS + 1));
    tmp.dsort_words = (uint32_t*)take(sort_words_bytes(L.n_views, mcd));
    tmp.max_dchunks = mcd;
    tmp.tstable = (uint32_t*)take(sizeof(uint32_t) * 4 * (GS_MAX_VIEWS + 1));
    tmp.max_ts_chunks = (capacity + kTsChunk - 1) / kTsChunk + L.n_views;
    const int mt = max_view_tiles(L);
    tmp.ts_len = mt <= kTsBins ? (int64_t)mt * tmp.max_ts_chunks : 0;
    tmp.tsm = (uint32_t*)take(sizeof(uint32_t) * (size_t)(tmp.ts_len + 1));
    tmp.ts_sums = (uint64_t*)take(sizeof(uint64_t) * (size_t)(tmp.ts_len / kScanBlock + 2));
    if (w) *w = tmp;
    return off;
}

size_t bin_sort_workspace(int64_t n, const gs_layout& L, int64_t capacity) {
    return carve(n, L, capacity, nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// generic exclusive scan of uint32 -> uint32 (64-bit carries)
// ---------------------------------------------------------------------------

GS_DEV uint64_t block_reduce_u64(uint64_t v, uint64_t* lds) {
    // wave reduction with shuffles, then across the 4 waves
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) t += lds[i];
    __syncthreads();
    return t;
}

// inclusive scan across the block of one value per thread; returns inclusive
GS_DEV uint64_t block_scan_u64(uint64_t v, uint64_t* lds, uint64_t* total) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    uint64_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint64_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == kWave - 1) lds[w] = x;
    __syncthreads();
    const int nw = blockDim.x / kWave;
    uint64_t pre = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) pre += lds[i];
        tot += lds[i];
    }
    __syncthreads();
    *total = tot;
    return x + pre;
}

// With `perm`, element i of the sequence is in[perm[i]], and the exclusive
// scan value of element i is stored as out[perm[i]] = scan_i (minus
// sub[perm[i]] if sub is set; no total is stored); without, element i is
// in[i] and out[i] = scan_i, with the total in out[len].
// `clear`, if set, is zeroed by the first launch (the status word of the call).
struct ScanIO {
    const uint32_t* in;
    const uint32_t* perm;
    const uint32_t* sub;
    uint32_t* out;
    uint32_t* clear;
};

// Tile rows of the bounding box in a projection record (rect0, rect1 words).
GS_DEV uint32_t rect_rows(const float4& q3) {
    return (__float_as_uint(q3.y) >> 16) - (__float_as_uint(q3.x) >> 16);
}

GS_DEV uint32_t scan_load(const ScanIO& io, int64_t i) { return io.perm ? io.in[io.perm[i]] : io.in[i]; }
GS_DEV void scan_store(const ScanIO& io, int64_t i, uint32_t x) {
    if (io.perm) {
        const uint32_t j = io.perm[i];
        io.out[j] = io.sub ? x - io.sub[j] : x;
    } else {
        io.out[i] = x;
    }
}

// A block's kScanBlock elements, kScanItems consecutive per thread: loaded
// (two 16-byte loads per thread when the block is whole and the arrays are
// 16-byte aligned, which the direct, in-order case allows), scanned across the
// block from `carry`, and stored.  Returns the block's total in *tot.
static_assert(kScanItems == 8, "two 16-byte vectors per thread");
GS_DEV void scan_block(const ScanIO& io, int64_t len, int64_t base, uint64_t carry, uint64_t* lds,
                       uint64_t* tot) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kScanItems;
    const bool vec = !io.perm && base + kScanBlock <= len &&
                     ((reinterpret_cast<uintptr_t>(io.in) | reinterpret_cast<uintptr_t>(io.out)) & 15u) == 0;
    uint32_t v[kScanItems];
    if (vec) {
        const uint4 a = reinterpret_cast<const uint4*>(io.in + i0)[0];
        const uint4 b = reinterpret_cast<const uint4*>(io.in + i0)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) v[i] = i0 + i < len ? scan_load(io, i0 + i) : 0u;
    }
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) s += v[i];
    const uint64_t inc = block_scan_u64(s, lds, tot);
    uint64_t run = carry + inc - s;
    uint32_t o[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        o[i] = (uint32_t)run;
        run += v[i];
    }
    if (vec) {
        reinterpret_cast<uint4*>(io.out + i0)[0] = make_uint4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<uint4*>(io.out + i0)[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
        for (int i = 0; i < kScanItems; ++i)
            if (i0 + i < len) scan_store(io, i0 + i, o[i]);
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(ScanIO io, int64_t len,
                                                              uint64_t* __restrict__ sums) {
    __shared__ uint64_t lds[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const int64_t idx = base + (int64_t)i * kScanThreads + threadIdx.x;
        if (idx < len) s += scan_load(io, idx);
    }
    if (io.clear && blockIdx.x == 0 && threadIdx.x == 0) *io.clear = 0u;
    s = block_reduce_u64(s, lds);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// single workgroup: exclusive scan of nb block sums in place; sums[nb] = total
__global__ __launch_bounds__(1024) void k_scan_top(uint64_t* __restrict__ sums, int64_t nb,
                                                   uint32_t* __restrict__ status) {
    __shared__ uint64_t lds[1024 / kWave];
    uint64_t carry = 0;
    for (int64_t b = 0; b < nb; b += 1024) {
        const int64_t i = b + threadIdx.x;
        const uint64_t v = i < nb ? sums[i] : 0;
        uint64_t tot;
        const uint64_t inc = block_scan_u64(v, lds, &tot);
        if (i < nb) sums[i] = carry + inc - v;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        sums[nb] = carry;
        if (status && carry > 0xFFFFFFFFull) atomicOr(status, (uint32_t)GS_STATUS_OVERFLOW);
    }
}

// `in` and `out` may be the same array.
__global__ __launch_bounds__(kScanThreads) void k_scan_down(ScanIO io, int64_t len,
                                                            const uint64_t* __restrict__ sums,
                                                            int64_t nb) {
    __shared__ uint64_t lds[kScanThreads / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint64_t tot;
    scan_block(io, len, base, sums[blockIdx.x], lds, &tot);
    if (!io.perm && blockIdx.x == 0 && threadIdx.x == 0) io.out[len] = (uint32_t)sums[nb];
}

// Second pass of a two-launch scan (for at most kScanInlineBlocks blocks):
// each block adds up the block sums before it itself, instead of a separate
// scan of the block sums; the last block writes the total.
constexpr int64_t kScanInlineBlocks = 2048;

__global__ __launch_bounds__(kScanThreads) void k_scan_down_inline(ScanIO io, int64_t len,
                                                                   const uint64_t* __restrict__ sums,
                                                                   int64_t nb,
                                                                   uint32_t* __restrict__ status) {
    __shared__ uint64_t lds[kScanThreads / kWave];
    uint64_t carry = 0;
    for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kScanThreads) carry += sums[i];
    carry = block_reduce_u64(carry, lds);
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    uint64_t tot;
    scan_block(io, len, base, carry, lds, &tot);
    if (blockIdx.x == nb - 1 && threadIdx.x == 0) {
        const uint64_t total = carry + tot;
        if (!io.perm) io.out[len] = (uint32_t)total;
        if (status && total > 0xFFFFFFFFull) atomicOr(status, (uint32_t)GS_STATUS_OVERFLOW);
    }
}

static int scan_exclusive(const uint32_t* in, int64_t len, uint32_t* out, uint64_t* sums,
                          uint32_t* status, hipStream_t s, const uint32_t* perm = nullptr,
                          const uint32_t* sub = nullptr, uint32_t* clear = nullptr) {
    const ScanIO io{in, perm, sub, out, clear};
    const int64_t nb = std::max<int64_t>((len + kScanBlock - 1) / kScanBlock, 1);
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, io, len, sums);
    if (nb <= kScanInlineBlocks) {
        hipLaunchKernelGGL(k_scan_down_inline, dim3((unsigned)nb), dim3(kScanThreads), 0, s, io, len, sums, nb,
                           status);
        return check_launch("scan");
    }
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, sums, nb, status);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, io, len, sums, nb);
    return check_launch("scan");
}

// ---------------------------------------------------------------------------
// per-view segment table
// ---------------------------------------------------------------------------

// Also clears the tile sort's digit totals.
// Tiles of each view (for the single-pass tile scatter).
struct TsGeom {
    int32_t ntiles[GS_MAX_VIEWS];
    int32_t tile_base[GS_MAX_VIEWS + 1];
    int32_t depth_bits[GS_MAX_VIEWS];
};

// With tstable: the tile scatter's chunks of kTsChunk keys per view, and the
// base of each view's tiles x chunks count matrix (views in order, each
// tile-major), whose total length goes to tstable[4 * n_views + 1].
__global__ void k_view_table(const uint32_t* __restrict__ offsets, int64_t n, int n_views,
                             int64_t capacity, uint32_t* __restrict__ table,
                             uint32_t* __restrict__ status, uint32_t* __restrict__ dcount,
                             uint32_t* __restrict__ tstable, TsGeom tg) {
    for (int i = threadIdx.x; i < n_views * kPasses * kDigits; i += blockDim.x) dcount[i] = 0u;
    if (threadIdx.x != 0) return;
    uint32_t chunks = 0, tchunks = 0, mlen = 0;
    const uint64_t cap = (uint64_t)capacity;
    for (int v = 0; v < n_views; ++v) {
        uint64_t b = offsets[(int64_t)v * n], e = offsets[(int64_t)(v + 1) * n];
        b = b < cap ? b : cap;
        e = e < cap ? e : cap;
        const uint32_t nc = (uint32_t)((e - b + kChunk - 1) / kChunk);
        table[4 * v + 0] = (uint32_t)b;
        table[4 * v + 1] = (uint32_t)e;
        table[4 * v + 2] = chunks;
        table[4 * v + 3] = nc;
        chunks += nc;
        if (tstable) {
            const uint32_t tc = (uint32_t)((e - b + kTsChunk - 1) / kTsChunk);
            tstable[4 * v + 0] = tchunks;
            tstable[4 * v + 1] = tc;
            tstable[4 * v + 2] = mlen;
            tstable[4 * v + 3] = (uint32_t)tg.ntiles[v];
            tchunks += tc;
            mlen += tc * (uint32_t)tg.ntiles[v];
        }
    }
    table[4 * n_views] = chunks;
    if (tstable) {
        tstable[4 * n_views] = tchunks;
        tstable[4 * n_views + 1] = mlen;
    }
    if ((uint64_t)offsets[(int64_t)n_views * n] > cap) atomicOr(status, (uint32_t)GS_STATUS_CAPACITY);
}

// ---------------------------------------------------------------------------
// tile rows and key emission
// ---------------------------------------------------------------------------

struct EmitGeom {
    int32_t tiles_x[GS_MAX_VIEWS];
    int32_t tiles_y[GS_MAX_VIEWS];
    int32_t depth_bits[GS_MAX_VIEWS];
    int32_t split[GS_MAX_VIEWS];   // key bits (all depth bits) sorted in the depth order
    int32_t tile;
    int32_t cull;
};

// The first kernel of a call: clears the status word; per (view, Gaussian)
// its tile rows (the rows of its bounding box) and, for the depth order, the
// low split bits of its keys (depth bits only) with its index;
// workgroup 0 also writes the depth sort's table (one segment of n per view)
// and clears its digit totals.
__global__ __launch_bounds__(256) void k_row_count(const float4* __restrict__ rec,
                                                   const uint32_t* __restrict__ tiles, int64_t n,
                                                   int64_t m, EmitGeom geo, uint32_t* __restrict__ row_count,
                                                   uint32_t* __restrict__ status, uint32_t* __restrict__ dkey,
                                                   uint32_t* __restrict__ dval, uint32_t* __restrict__ dtable,
                                                   uint32_t* __restrict__ ddcount, int n_views,
                                                   bool depth_keys) {
    if (blockIdx.x == 0) {
        for (int i = threadIdx.x; i < n_views * kPasses * kDigits; i += blockDim.x) ddcount[i] = 0u;
        if (threadIdx.x == 0) {
            *status = 0u;
            const uint32_t dnc = (uint32_t)((n + kDepthChunk - 1) / kDepthChunk);
            for (int v = 0; v < n_views; ++v) {
                dtable[4 * v + 0] = (uint32_t)(v * n);
                dtable[4 * v + 1] = (uint32_t)((v + 1) * n);
                dtable[4 * v + 2] = (uint32_t)v * dnc;
                dtable[4 * v + 3] = dnc;
            }
            dtable[4 * n_views] = (uint32_t)n_views * dnc;
        }
    }
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= m) return;
    const bool vis = tiles[o] > 0;
    // records of Gaussians outside the view are not read
    const float4 q3 = vis ? rec[4 * o + 3] : make_float4(0.f, 0.f, 0.f, 0.f);
    row_count[o] = vis ? rect_rows(q3) : 0u;
    if (!depth_keys) return;   // no depth order in this call
    const int v = (int)(o / n);
    // the key's bits below split (at most D): depth bits only
    const int D = geo.depth_bits[v];
    const int split = geo.split[v];
    const uint32_t dk = __float_as_uint(q3.z) >> (23 - D);
    dkey[o] = vis ? dk & ((1u << split) - 1u) : 0u;
    dval[o] = (uint32_t)o;
}

// One thread per (view, Gaussian): the column span of each of its tile rows
// (the rectangle's columns, or the ellipse's span of that row), recorded as
// the unsorted index of the row's first tile and its first column, with the
// Gaussian's depth bits.  The spans are the ones the projection counted (same
// function of the same record values).
__global__ __launch_bounds__(256) void k_rows(const float4* __restrict__ rec,
                                              const uint32_t* __restrict__ tiles,
                                              const uint32_t* __restrict__ offsets,
                                              const uint32_t* __restrict__ row_offsets, int64_t n,
                                              int64_t m, EmitGeom geo, int64_t row_capacity,
                                              uint4* __restrict__ rows, uint32_t* __restrict__ status) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= m || tiles[o] == 0) return;
    const int v = (int)(o / n);
    const float4* r = rec + 4 * o;
    const float4 q0 = r[0], q1 = r[1], q3 = r[3];
    const uint32_t r0 = __float_as_uint(q3.x), r1 = __float_as_uint(q3.y);
    const int x0 = (int)(r0 & 0xFFFF), y0 = (int)(r0 >> 16), x1 = (int)(r1 & 0xFFFF), y1 = (int)(r1 >> 16);
    Ellipse e;
    const bool ell = geo.cull == GS_CULL_ELLIPSE;
    if (ell) ellipse_setup(q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, e);
    uint32_t first = offsets[o];
    const uint32_t dk = __float_as_uint(q3.z) >> (23 - geo.depth_bits[v]);
    const uint64_t rs = row_offsets[o];
    if (rs + (uint64_t)(y1 - y0) > (uint64_t)row_capacity) atomicOr(status, (uint32_t)GS_STATUS_ROWS);
    for (int ty = y0; ty < y1; ++ty) {
        int xa = x0, xb = x1;
        if (ell) ellipse_span(e, geo.tile, geo.tiles_x[v], ty, xa, xb);
        if (xb < xa) xb = xa;
        const uint64_t slot = rs + (uint64_t)(ty - y0);
        if (slot < (uint64_t)row_capacity)
            rows[slot] = make_uint4(first, (uint32_t)o, (uint32_t)xa | ((uint32_t)ty << 16), dk);
        first += (uint32_t)(xb - xa);
    }
}

constexpr int kEmitG = 256;  // tile rows per workgroup

// A workgroup owns kEmitG consecutive row slots.  Their first indices, tile
// bases and depth codes are staged in LDS; the workgroup's intersections
// [rows[r0].first, rows[r0 + kEmitG].first) are then produced by consecutive
// threads (balanced however unequal the rows are), each finding its row by
// binary search over the staged first indices.  With `dpos` (each
// (view, Gaussian)'s first position in depth order) each key goes to its
// unsorted index minus its Gaussian's first unsorted index plus that
// position, so that the keys of a view are laid out by (depth bits,
// Gaussian id).
__global__ __launch_bounds__(kEmitG) void k_emit(const float4* __restrict__ rec,
                                                 const uint4* __restrict__ rows,
                                                 const uint32_t* __restrict__ row_offsets,
                                                 const uint32_t* __restrict__ offsets,
                                                 const uint32_t* __restrict__ dpos, int64_t n,
                                                 int64_t m, EmitGeom geo, int64_t capacity,
                                                 int64_t row_capacity, uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals) {
    __shared__ uint32_t s_off[kEmitG + 1];
    __shared__ uint32_t s_tile[kEmitG];   // tile index (within the view) of the row's first tile
    __shared__ uint32_t s_dk[kEmitG];     // depth bits
    __shared__ uint32_t s_gid[kEmitG];
    __shared__ uint32_t s_sh[kEmitG];     // depth-order position minus unsorted index
    __shared__ uint8_t s_D[kEmitG];
    const uint64_t kc = min((uint64_t)offsets[m], (uint64_t)capacity);
    const uint64_t rc = min((uint64_t)row_offsets[m], (uint64_t)row_capacity);
    const uint64_t r0 = (uint64_t)blockIdx.x * kEmitG;
    if (r0 >= rc) return;
    const int t = threadIdx.x;
    const uint64_t r = r0 + (uint64_t)t;
    if (r < rc) {
        const uint4 row = rows[r];
        s_off[t] = (uint32_t)min((uint64_t)row.x, kc);
        const int64_t o = (int64_t)row.y;
        const int v = (int)(o / n);
        const int D = geo.depth_bits[v];
        s_tile[t] = (row.z >> 16) * (uint32_t)geo.tiles_x[v] + (row.z & 0xFFFF);
        s_dk[t] = row.w;
        s_gid[t] = (uint32_t)(o - (int64_t)v * n);
        s_sh[t] = dpos ? dpos[o] - offsets[o] : 0u;
        s_D[t] = (uint8_t)D;
    } else {
        s_off[t] = (uint32_t)kc;
        s_tile[t] = 0; s_dk[t] = 0; s_gid[t] = 0; s_sh[t] = 0; s_D[t] = 0;
    }
    if (t == 0) s_off[kEmitG] = r0 + kEmitG < rc ? (uint32_t)min((uint64_t)rows[r0 + kEmitG].x, kc) : (uint32_t)kc;
    __syncthreads();
    const uint32_t begin = s_off[0], end = s_off[kEmitG];
    for (uint64_t i = (uint64_t)begin + t; i < end; i += kEmitG) {
        int lo = 0, hi = kEmitG - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= i) lo = mid; else hi = mid - 1;
        }
        const uint32_t tile = s_tile[lo] + (uint32_t)(i - s_off[lo]);
        const uint32_t pos = (uint32_t)i + s_sh[lo];   // shift 0 without the depth order
        if ((uint64_t)pos < kc) {
            keys[pos] = (tile << s_D[lo]) | s_dk[lo];
            vals[pos] = s_gid[lo];
        }
    }
}

// ---------------------------------------------------------------------------
// radix sort: one histogram pass for all four digits, then one single-pass
// scatter per digit whose global destinations come from a decoupled look-back
// over the preceding chunks of the same view
// ---------------------------------------------------------------------------

// Chunk b -> (view, chunk within view).  Returns false for unused chunks.
GS_DEV bool chunk_of(const uint32_t* table, int n_views, uint32_t b, int* view, uint32_t* c) {
    if (b >= table[4 * n_views]) return false;
    int v = 0;
    for (int i = 0; i < n_views; ++i)
        if (table[4 * i + 3] > 0 && b >= table[4 * i + 2]) v = i;
    *view = v;
    *c = b - table[4 * v + 2];
    return true;
}

// Look-back words: flag in the high half, a count in the low half.
constexpr uint64_t kLbAggregate = 1ull << 32;  // count of this chunk (or group) alone
constexpr uint64_t kLbPrefix = 2ull << 32;     // count of this chunk and all before it in the view
constexpr uint32_t kLbSpinLimit = 1u << 20;

struct SortWs {
    uint32_t* dcount;   // [n_views][kPasses][kDigits] digit totals (cleared by the table kernel)
    uint64_t* agg;      // [kPasses][max_chunks][kDigits] kLbAggregate | chunk count
    uint64_t* pre;      // [kPasses][max_chunks][kDigits] kLbPrefix | inclusive prefix
    uint64_t* gagg;     // [kPasses][max_groups][kDigits] kLbAggregate | group count
    uint32_t* gdone;    // [kPasses][max_groups] chunks of the group that have published
    int64_t max_chunks;
    int64_t max_groups;
    int32_t passes;                  // digits sorted (1..kPasses), least significant first
    int32_t shift0[GS_MAX_VIEWS];    // bit position of each view's first digit
};

// Digit of `key` for a pass whose digit starts at bit `shift` (bits past 31
// read as zero).
GS_DEV uint32_t digit_at(uint32_t key, int shift) { return shift < 32 ? (key >> shift) & 0xFFu : 0u; }

static SortWs carve_sort(void* base, int n_views, int64_t mc) {
    SortWs S;
    const int64_t mg = max_groups_for(mc, n_views);
    const size_t nd = (size_t)n_views * kPasses * kDigits;
    char* p = (char*)base;
    S.dcount = (uint32_t*)p;
    p += align_up(4 * nd);
    S.agg = (uint64_t*)p;
    p += align_up(8 * (size_t)(kPasses * mc * kDigits));
    S.pre = (uint64_t*)p;
    p += align_up(8 * (size_t)(kPasses * mc * kDigits));
    S.gagg = (uint64_t*)p;
    p += align_up(8 * (size_t)(kPasses * mg * kDigits));
    S.gdone = (uint32_t*)p;
    S.max_chunks = mc;
    S.max_groups = mg;
    S.passes = kPasses;
    for (int v = 0; v < GS_MAX_VIEWS; ++v) S.shift0[v] = 0;
    return S;
}

// Look-back groups: kGroup consecutive chunks of a view.  Group (v, i) has
// slot floor(chunk_base_v / kGroup) + v + i, which is unique and below
// max_chunks / kGroup + n_views + 1.

GS_DEV uint32_t group_slot(const uint32_t* table, int v, uint32_t c) {
    return table[4 * v + 2] / kGroup + (uint32_t)v + c / kGroup;
}

// Digit totals of every pass, per view.  A grid-stride loop over chunks
// counts keys in per-wavefront LDS histograms and adds the non-zero totals to
// the view's when the view changes and at the end (few workgroups, so each
// total takes few global atomics).  Each chunk's look-back words, and its
// group's if it is the group's first chunk, are cleared for all passes.
template <int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_digit_hist(const uint32_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ table,
                                                             int n_views, SortWs S) {
    constexpr int NW = kSortThreads / kWave;
    __shared__ uint32_t cnt[NW][kPasses][kDigits];
    const int t = threadIdx.x, w = t / kWave;
    const uint32_t used = table[4 * n_views];
#pragma unroll
    for (int j = 0; j < NW * kPasses; ++j) (&cnt[0][0][0])[j * kDigits + t] = 0u;
    __syncthreads();
    int cur = -1;
    for (uint32_t b = blockIdx.x; b < used; b += gridDim.x) {
        int v;
        uint32_t c;
        chunk_of(table, n_views, b, &v, &c);
        if (cur >= 0 && v != cur) {
            __syncthreads();
#pragma unroll
            for (int p = 0; p < kPasses; ++p) {
                uint32_t x = 0;
#pragma unroll
                for (int j = 0; j < NW; ++j) {
                    x += cnt[j][p][t];
                    cnt[j][p][t] = 0u;
                }
                if (x && p < S.passes) atomicAdd(&S.dcount[(cur * kPasses + p) * kDigits + t], x);
            }
            __syncthreads();
        }
        cur = v;
        const uint32_t seg_e = table[4 * v + 1];
        const uint32_t start = table[4 * v] + c * (ITEMS * kSortThreads);
        uint32_t k[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = start + i * kSortThreads + t;
            k[i] = idx < seg_e ? keys[idx] : 0u;
        }
        const uint32_t gs = group_slot(table, v, c);
        const int sh0 = S.shift0[v];
        for (int p = 0; p < S.passes; ++p) {
            S.agg[((int64_t)p * S.max_chunks + b) * kDigits + t] = 0ull;
            S.pre[((int64_t)p * S.max_chunks + b) * kDigits + t] = 0ull;
            if (c % kGroup == 0) {
                S.gagg[((int64_t)p * S.max_groups + gs) * kDigits + t] = 0ull;
                if (t == 0) S.gdone[p * S.max_groups + gs] = 0u;
            }
        }
        // runs of equal digits in consecutive lanes (a Gaussian's keys share
        // their depth bits) are counted by their first lane: one LDS atomic per
        // run instead of one per key
        const int lane = t % kWave;
        const uint64_t above = lane == kWave - 1 ? 0ull : (~0ull << (lane + 1));
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = start + i * kSortThreads + t;
            const bool valid = idx < seg_e;
            const uint64_t vmask = __ballot(valid);
            const uint32_t prev = __shfl_up(k[i], 1);
#pragma unroll
            for (int p = 0; p < kPasses; ++p) {
                if (p >= S.passes) break;
                const uint32_t dg = digit_at(k[i], sh0 + 8 * p);
                const bool head = valid && (lane == 0 || digit_at(prev, sh0 + 8 * p) != dg);
                const uint64_t heads = __ballot(head) | ~vmask;   // invalid lanes end runs
                if (head) {
                    const uint64_t nxt = heads & above;
                    const int end = nxt ? __builtin_ctzll(nxt) : kWave;
                    atomicAdd(&cnt[w][p][dg], (uint32_t)(end - lane));
                }
            }
        }
    }
    __syncthreads();
    if (cur >= 0) {
#pragma unroll
        for (int p = 0; p < kPasses; ++p) {
            uint32_t x = 0;
#pragma unroll
            for (int j = 0; j < NW; ++j) x += cnt[j][p][t];
            if (x && p < S.passes) atomicAdd(&S.dcount[(cur * kPasses + p) * kDigits + t], x);
        }
    }
}

GS_DEV uint64_t lanemask_lt() {
    const int lane = threadIdx.x % kWave;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}


GS_DEV uint64_t lb_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

GS_DEV void lb_store(uint64_t* p, uint64_t x) {
    __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Polls a look-back word until its flag is set (or the spin limit is hit).
GS_DEV uint64_t lb_wait(const uint64_t* p, uint32_t* status) {
    uint64_t x = lb_load(p);
    for (uint32_t spins = 0; (x >> 32) == 0; ++spins) {
        if (spins > kLbSpinLimit) {
            atomicOr(status, (uint32_t)GS_STATUS_SORT);
            return kLbAggregate;
        }
        __builtin_amdgcn_s_sleep(1);
        x = lb_load(p);
    }
    return x;
}

constexpr int kLbGroupWindow = 8;

// A key's rank: its group's base, held by the group's first lane, plus its
// rank in the group (lead: that lane, then the rank, from bit 8).
GS_DEV uint32_t finish_rank(uint32_t base, uint32_t lead) {
    return (uint32_t)__shfl((int)base, (int)(lead & 0x3Fu)) + (lead >> 8);
}

// One stable radix pass over a chunk of 256 ITEMS keys; chunk b is workgroup b.
// Workgroups start in index order, and each publishes its per-digit counts
// before it waits on anything, so every wait of the look-back is on a chunk
// that has started and will publish; a spin limit bounds the waits all the
// same (GS_STATUS_SORT).
//
// Wavefront w owns the contiguous keys [w * PER_WAVE, (w + 1) * PER_WAVE) of the chunk
// and ranks them item by item: peers with the same digit are found with 8
// ballots, and a running per-(wavefront, digit) count in LDS gives each key its
// rank among the wavefront's keys of that digit (one wavefront updates only
// its own counts, so no barrier is needed while ranking).  A scan over
// (digit, wavefront) turns the counts into chunk-local positions, the keys are
// placed in LDS in digit order and written out so that consecutive lanes write
// consecutive addresses of each digit's run; then the values, read only now,
// take the same LDS buffer and go out the same way.  The order of equal digits
// is (chunk, wavefront, item, lane) = input order: stable.
//
// Destinations: the digit's start in the view plus the counts of the view's
// earlier chunks.  Each chunk publishes its count, and the chunk of a group of
// kGroup that publishes last also the group's total; a chunk then adds the
// counts of the earlier chunks of its group and the totals of the earlier
// groups, stopping early at the published inclusive prefix of a group's last
// chunk.
// With 6144-key chunks (runs of 24 keys per digit on average) one 24 KB
// buffer for keys and then values and at most 168 VGPRs let three workgroups
// share a CU: 2% faster on 1.6e8 keys than 8192-key chunks holding keys and
// values in LDS together (two per CU); 8192-key chunks with the one buffer
// spill at three per CU, and 6144 at four.  The depth sort of 3e5 (view, Gaussian)s
// runs 2048-key chunks: 1024 took 10% longer (more look-back groups), 4096
// 15% (fewer workgroups than CUs).
template <int ITEMS>
__global__ __launch_bounds__(kSortThreads) __attribute__((amdgpu_waves_per_eu(ITEMS >= 24 ? 3 : 4))) void k_onesweep(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out,
    const uint32_t* __restrict__ table, int n_views, int pass, SortWs S,
    uint32_t* __restrict__ status) {
    constexpr int NW = kSortThreads / kWave;
    constexpr int CHUNK = ITEMS * kSortThreads;
    constexpr int PER_WAVE = CHUNK / NW;
    constexpr int kLag = ITEMS < 4 ? ITEMS : 4;
    // global destination of the chunk's keys of digit d minus their
    // chunk-local start
    __shared__ uint32_t goff[kDigits];
    __shared__ uint32_t wcnt[NW][kDigits];
    // the chunk's keys in sorted order, then its values (and, while the
    // chunk is ranked, the target of the non-leading lanes' atomics)
    __shared__ uint32_t s_buf[CHUNK];
    __shared__ uint8_t s_dg[CHUNK];       // digit of each sorted position
    __shared__ uint64_t s_scan[NW];
    __shared__ uint32_t s_last;
    const uint32_t b = blockIdx.x;
    int v;
    uint32_t c;
    if (!chunk_of(table, n_views, b, &v, &c)) return;
    const int shift = S.shift0[v] + 8 * pass;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int j = 0; j < NW; ++j) wcnt[j][threadIdx.x] = 0u;
    const uint32_t seg_e = table[4 * v + 1];
    const uint32_t start = table[4 * v] + c * CHUNK;
    const uint32_t n_here = min((uint32_t)CHUNK, seg_e - start);
    // this lane's first key; its i-th is kWave * i further (one base address
    // and immediate offsets, not a live address per item)
    const uint32_t idx0 = start + w * PER_WAVE + lane;
    const uint32_t* __restrict__ kp = keys_in + idx0;
    uint32_t k[ITEMS], rank[ITEMS], lead[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) k[i] = idx0 + i * kWave < seg_e ? kp[i * kWave] : 0u;
    const uint64_t lt = lanemask_lt();
    // the view's total of this thread's digit (its start is their exclusive scan)
    const uint32_t dtot = S.dcount[(v * kPasses + pass) * kDigits + threadIdx.x];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = idx0 + i * kWave < seg_e;
        const uint32_t d = digit_at(k[i], shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (d >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint64_t before = peers & lt;
        // the first lane of each digit group takes the wavefront's count and
        // advances it in one LDS atomic; a wavefront's LDS operations complete
        // in issue order, so item i + 1's atomics need not wait for item i's
        // result.  Every lane issues the atomic, the others adding 0 to a
        // slot of their own: without a branch the compiler waits for each
        // result only where it is used.
        const bool first = valid && before == 0ull;
        rank[i] = atomicAdd(first ? &wcnt[w][d] : &s_buf[threadIdx.x], first ? (uint32_t)__popcll(peers) : 0u);
        lead[i] = valid ? (uint32_t)__builtin_ctzll(peers) | ((uint32_t)__popcll(before) << 8) : 0u;
        // every key's rank: its group's base from the group's first lane,
        // kLag items later (by then the atomic has returned)
        if (i >= kLag) rank[i - kLag] = finish_rank(rank[i - kLag], lead[i - kLag]);
    }
#pragma unroll
    for (int i = ITEMS - kLag; i < ITEMS; ++i) rank[i] = finish_rank(rank[i], lead[i]);
    __syncthreads();
    const uint32_t d = threadIdx.x;
    const int64_t cw = (int64_t)pass * S.max_chunks * kDigits;   // this pass's chunk words
    const int64_t gw = (int64_t)pass * S.max_groups * kDigits;   // this pass's group words
    const uint32_t nc = table[4 * v + 3];
    const uint32_t gi = c / kGroup, g0 = b - c % kGroup;         // group, its first chunk
    uint32_t total = 0;
#pragma unroll
    for (int j = 0; j < NW; ++j) total += wcnt[j][d];
    lb_store(&S.agg[cw + (int64_t)b * kDigits + d], kLbAggregate | total);
    if (c == 0) lb_store(&S.pre[cw + (int64_t)b * kDigits + d], kLbPrefix | total);
    if (d == 0) {
        const uint32_t gsize = min((uint32_t)kGroup, nc - gi * kGroup);
        s_last = atomicAdd(&S.gdone[pass * S.max_groups + group_slot(table, v, c)], 1u) + 1 == gsize;
    }
    uint32_t dbase, lstart;
    {
        // digit-major exclusive scan over (digit, wavefront), and in the high
        // half the exclusive scan of the view's digit totals (no carry: the
        // chunk's counts sum to at most CHUNK)
        uint64_t tot;
        const uint64_t both = ((uint64_t)dtot << 32) | total;
        const uint64_t inc = block_scan_u64(both, s_scan, &tot);
        dbase = table[4 * v] + (uint32_t)((inc - both) >> 32);
        uint32_t run = (uint32_t)(inc - both);
        lstart = run;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const uint32_t x = wcnt[j][d];
            wcnt[j][d] = run;
            run += x;
        }
    }
    __syncthreads();
    // keys to their chunk-local sorted positions (rank[] becomes the position)
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = start + w * PER_WAVE + i * kWave + lane;
        if (idx < seg_e) {
            const uint32_t dg = digit_at(k[i], shift);
            rank[i] += wcnt[w][dg];
            s_buf[rank[i]] = k[i];
            s_dg[rank[i]] = (uint8_t)dg;
        }
    }
    if (s_last) {
        // last of its group to publish: every chunk of the group has stored its
        // count (its flag may still be in flight, so poll it)
        const uint32_t gsize = min((uint32_t)kGroup, nc - gi * kGroup);
        uint64_t x[kGroup];
#pragma unroll
        for (int j = 0; j < kGroup; ++j)
            x[j] = (uint32_t)j < gsize ? lb_load(&S.agg[cw + (int64_t)(g0 + j) * kDigits + d]) : kLbAggregate;
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < kGroup; ++j) {
            if ((x[j] >> 32) == 0) x[j] = lb_wait(&S.agg[cw + (int64_t)(g0 + j) * kDigits + d], status);
            sum += (uint32_t)x[j];
        }
        lb_store(&S.gagg[gw + (int64_t)group_slot(table, v, c) * kDigits + d], kLbAggregate | sum);
    }
    // look-back, one digit per thread
    uint32_t excl = 0;
    if (c > 0) {
        bool done = false;
        // counts of the earlier chunks of the own group, all loads at once
        const uint32_t cin = b - g0;
        uint64_t aj[kGroup - 1];
#pragma unroll
        for (int q = 0; q < kGroup - 1; ++q)
            aj[q] = (uint32_t)q < cin ? lb_load(&S.agg[cw + ((int64_t)g0 + q) * kDigits + d]) : kLbAggregate;
#pragma unroll
        for (int q = 0; q < kGroup - 1; ++q) {
            if ((aj[q] >> 32) == 0) aj[q] = lb_wait(&S.agg[cw + ((int64_t)g0 + q) * kDigits + d], status);
            excl += (uint32_t)aj[q];
        }
        // earlier groups, kLbGroupWindow per round: the inclusive prefix of a
        // group's last chunk ends the walk, else the group's total is added
        int64_t g = (int64_t)gi - 1;
        const uint32_t slot0 = group_slot(table, v, 0);
        while (!done && g >= 0) {
            uint64_t pl[kLbGroupWindow], ga[kLbGroupWindow];
#pragma unroll
            for (int q = 0; q < kLbGroupWindow; ++q) {
                const int64_t gq = g - q;
                const uint32_t last = b - c + (uint32_t)gq * kGroup + (kGroup - 1);
                pl[q] = gq >= 0 ? lb_load(&S.pre[cw + (int64_t)last * kDigits + d]) : kLbPrefix;
                ga[q] = gq >= 0 ? lb_load(&S.gagg[gw + (int64_t)(slot0 + gq) * kDigits + d]) : 0ull;
            }
            int used = 0;
            bool stall = false;
#pragma unroll
            for (int q = 0; q < kLbGroupWindow; ++q) {
                if (!done && !stall) {
                    if (pl[q] >> 32) {
                        excl += (uint32_t)pl[q];
                        done = true;
                    } else if (ga[q] >> 32) {
                        excl += (uint32_t)ga[q];
                        ++used;
                    } else {
                        stall = true;
                    }
                }
            }
            g -= used;
            if (stall && !done) {
                // the group's total is not out yet: wait for it
                excl += (uint32_t)lb_wait(&S.gagg[gw + (int64_t)(slot0 + g) * kDigits + d], status);
                --g;
            }
        }
        lb_store(&S.pre[cw + (int64_t)b * kDigits + d], kLbPrefix | (excl + total));
    }
    goff[d] = dbase + excl - lstart;
    // the values, read in input order while the keys go out
    const uint32_t* __restrict__ vp = vals_in + idx0;
    uint32_t val[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) val[i] = idx0 + i * kWave < seg_e ? vp[i * kWave] : 0u;
    __syncthreads();
    // keys out: consecutive lanes write consecutive addresses of each digit's run
    for (uint32_t j = threadIdx.x; j < n_here; j += kSortThreads) {
        const uint32_t key = s_buf[j];
        keys_out[j + goff[digit_at(key, shift)]] = key;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if (idx0 + i * kWave < seg_e) s_buf[rank[i]] = val[i];
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < n_here; j += kSortThreads) vals_out[j + goff[s_dg[j]]] = s_buf[j];
}

// Stable sort of each view's segment of (keys, vals) by S.passes 8-bit digits
// starting at bit S.shift0[view], through (ktmp, vtmp).  `table` describes the
// segments and chunks; dcount must be zero.
template <int ITEMS>
static int radix_sort_views(uint32_t* keys, uint32_t* vals, uint32_t* ktmp, uint32_t* vtmp,
                            const uint32_t* table, int n_views, const SortWs& S, uint32_t* status,
                            hipStream_t s) {
    int rc;
    const unsigned hgrid = (unsigned)std::min<int64_t>(S.max_chunks, kHistBlocks);
    hipLaunchKernelGGL(k_digit_hist<ITEMS>, dim3(hgrid), dim3(kSortThreads), 0, s, keys, table, n_views, S);
    if ((rc = check_launch("digit_hist")) != GS_OK) return rc;
    // an even number of passes leaves the result in keys / vals, an odd
    // number in ktmp / vtmp
    uint32_t *kin = keys, *vin = vals, *kout = ktmp, *vout = vtmp;
    for (int pass = 0; pass < S.passes; ++pass) {
        hipLaunchKernelGGL(k_onesweep<ITEMS>, dim3((unsigned)S.max_chunks), dim3(kSortThreads), 0, s, kin, vin, kout,
                           vout, table, n_views, pass, S, status);
        if ((rc = check_launch("onesweep")) != GS_OK) return rc;
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return GS_OK;
}

// ---------------------------------------------------------------------------
// tile ranges
// ---------------------------------------------------------------------------

struct RangeGeom {
    int32_t depth_bits[GS_MAX_VIEWS];
    int32_t tiles_x[GS_MAX_VIEWS];
    int32_t tile_base[GS_MAX_VIEWS + 1];
};

// Tile boundaries -> ranges (lower-bound semantics, empty tiles get start =
// end = insertion point): a grid-stride loop in which each thread takes four
// consecutive sorted positions (one 16-byte load and the key before them);
// one workgroup per 256 positions was bound by the workgroup dispatch rate at
// 10^8 keys.  Then the same threads give the tiles of views without any
// intersection their empty range.
constexpr int kRangeBlocks = 16384;

GS_DEV void range_bounds(uint2* R, int nt, uint32_t j, int t, int tp, bool first, bool last) {
    if (first) {
        for (int u = 0; u <= t; ++u) R[u].x = j;
        for (int u = 0; u < t; ++u) R[u].y = j;
    } else if (tp != t) {
        for (int u = tp + 1; u <= t; ++u) R[u].x = j;
        for (int u = tp; u < t; ++u) R[u].y = j;
    }
    if (last) {
        for (int u = t; u < nt; ++u) R[u].y = j + 1;
        for (int u = t + 1; u < nt; ++u) R[u].x = j + 1;
    }
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ keys,
                                                const uint32_t* __restrict__ table, int n_views,
                                                RangeGeom geo, uint32_t* __restrict__ ranges) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t total = table[4 * (n_views - 1) + 1];   // the views' segments are consecutive
    for (int64_t q = first; 4 * q < (int64_t)total; q += stride) {
        const uint32_t j0 = (uint32_t)(4 * q);
        uint32_t k[4];
        if (j0 + 4 <= total) {
            const uint4 x = reinterpret_cast<const uint4*>(keys)[q];
            k[0] = x.x; k[1] = x.y; k[2] = x.z; k[3] = x.w;
        } else {
            for (int u = 0; u < 4; ++u) k[u] = j0 + u < total ? keys[j0 + u] : 0u;
        }
        const uint32_t kp = j0 > 0 ? keys[j0 - 1] : 0u;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t j = j0 + (uint32_t)u;
            if (j >= total) break;
            int v = 0;
            for (int i = 1; i < n_views; ++i)
                if (j >= table[4 * i]) v = i;
            const uint32_t sb = table[4 * v], se = table[4 * v + 1];
            const int D = geo.depth_bits[v];
            const int tb = geo.tile_base[v];
            const int nt = geo.tile_base[v + 1] - tb;
            const int t = min((int)(k[u] >> D), nt - 1);
            const int tp = j == sb ? 0 : min((int)((u > 0 ? k[u - 1] : kp) >> D), nt - 1);
            range_bounds(reinterpret_cast<uint2*>(ranges) + tb, nt, j, t, tp, j == sb, j == se - 1);
        }
    }
    for (int64_t gt = first; gt < (int64_t)geo.tile_base[n_views]; gt += stride) {
        int v = 0;
        for (int i = 1; i < n_views; ++i)
            if (gt >= geo.tile_base[i]) v = i;
        const uint32_t b = table[4 * v], e = table[4 * v + 1];
        if (b == e) reinterpret_cast<uint2*>(ranges)[gt] = make_uint2(b, b);
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

int launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s) {
    if (count <= 0) return GS_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, value,
                       count);
    return check_launch("fill");
}

// ---------------------------------------------------------------------------
// stand-alone stable sort of (key, value) pairs, one segment [0, count)
// ---------------------------------------------------------------------------

// Table of one segment [0, count); clears the digit totals.
__global__ void k_single_table(uint32_t* table, int64_t count, uint32_t* dcount, uint32_t* status) {
    for (int i = threadIdx.x; i < kPasses * kDigits; i += blockDim.x) dcount[i] = 0u;
    if (threadIdx.x != 0) return;
    table[0] = 0u;
    table[1] = (uint32_t)count;
    table[2] = 0u;
    table[3] = (uint32_t)((count + kChunk - 1) / kChunk);
    table[4] = table[3];
    *status = 0u;
}

struct PairsScratch {
    uint32_t *ktmp, *vtmp, *table, *status, *sort_words;
    int64_t mc;
};

static size_t carve_pairs(int64_t count, char* base, PairsScratch* out) {
    PairsScratch P;
    P.mc = (count + kChunk - 1) / kChunk + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    P.ktmp = (uint32_t*)take(4 * (size_t)count);
    P.vtmp = (uint32_t*)take(4 * (size_t)count);
    P.table = (uint32_t*)take(4 * 8);
    P.status = (uint32_t*)take(4);
    P.sort_words = (uint32_t*)take(sort_words_bytes(1, P.mc));
    if (out) *out = P;
    return off;
}

size_t sort_pairs_scratch(int64_t count) { return carve_pairs(count, nullptr, nullptr); }

int sort_pairs(uint32_t* keys, uint32_t* vals, int64_t count, void* scratch, hipStream_t s) {
    if (count <= 1) return GS_OK;
    PairsScratch P;
    carve_pairs(count, (char*)scratch, &P);
    const SortWs S = carve_sort(P.sort_words, 1, P.mc);
    hipLaunchKernelGGL(k_single_table, dim3(1), dim3(256), 0, s, P.table, count, S.dcount, P.status);
    int rc = check_launch("sort_table");
    if (rc != GS_OK) return rc;
    return radix_sort_views<kSortItems>(keys, vals, P.ktmp, P.vtmp, P.table, 1, S, P.status, s);
}

// ---------------------------------------------------------------------------
// single-pass tile scatter: with the keys already in depth order, a stable
// partition by tile finishes the sort.  Chunks of kTsChunk consecutive keys
// count their tiles (a tiles x chunks matrix per view, tile-major); one
// exclusive scan of all the matrices in order gives, for every (view, tile,
// chunk), the sorted position of the chunk's first key of that tile (the
// view's segment start, plus the view's keys of earlier tiles, plus the
// tile's keys in earlier chunks); each chunk then ranks its keys within the
// chunk and writes them there.
// ---------------------------------------------------------------------------

// Workgroup -> chunk of the tile scatter, then (view, chunk within view).
// Workgroups are dealt to the 8 XCDs in turn, so XCD x is given the
// contiguous chunks [x * per, (x + 1) * per): consecutive chunks write
// neighbouring positions of every tile's run and count-matrix words of the
// same lines, which then meet in one L2 instead of eight.
GS_DEV bool ts_chunk_of(const uint32_t* tstable, int n_views, uint32_t wg, int* view, uint32_t* c) {
    const uint32_t total = tstable[4 * n_views];
    const uint32_t per = (total + 7u) / 8u;
    const uint32_t b = (wg % 8u) * per + wg / 8u;
    if (wg / 8u >= per || b >= total) return false;
    int v = 0;
    for (int i = 0; i < n_views; ++i)
        if (tstable[4 * i + 1] > 0 && b >= tstable[4 * i]) v = i;
    *view = v;
    *c = b - tstable[4 * v];
    return true;
}

// Per chunk: its keys per tile, into column c of its view's matrix.
// Workgroup 0 also writes the (empty) ranges of views without keys.
__global__ __launch_bounds__(kTsThreads) void k_ts_count(const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ table,
                                                         const uint32_t* __restrict__ tstable, int n_views,
                                                         TsGeom tg, uint32_t* __restrict__ tsm,
                                                         uint32_t* __restrict__ ranges) {
    __shared__ uint32_t hist[kTsBins];
    const int t = threadIdx.x;
    if (blockIdx.x == 0) {
        for (int v = 0; v < n_views; ++v) {
            if (tstable[4 * v + 1] != 0) continue;
            const uint32_t b = table[4 * v];
            for (int j = t; j < tg.ntiles[v]; j += kTsThreads)
                reinterpret_cast<uint2*>(ranges)[tg.tile_base[v] + j] = make_uint2(b, b);
        }
    }
    int v;
    uint32_t c;
    if (!ts_chunk_of(tstable, n_views, blockIdx.x, &v, &c)) return;
    const int nt = tg.ntiles[v], D = tg.depth_bits[v];
    for (int j = t; j < nt; j += kTsThreads) hist[j] = 0u;
    __syncthreads();
    const uint32_t seg_e = table[4 * v + 1];
    const uint32_t start = table[4 * v] + c * kTsChunk;
    // loads unconditional (clamped into the chunk), 8 in flight per lane
    for (int i0 = 0; i0 < kTsItems; i0 += 8) {
        uint32_t k[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) k[u] = keys[min(start + (uint32_t)((i0 + u) * kTsThreads + t), seg_e - 1)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (start + (uint32_t)((i0 + u) * kTsThreads + t) < seg_e)
                atomicAdd(&hist[min((int)(k[u] >> D), nt - 1)], 1u);
    }
    __syncthreads();
    const uint32_t nc = tstable[4 * v + 1], mb = tstable[4 * v + 2];
    for (int j = t; j < nt; j += kTsThreads) tsm[mb + (uint32_t)j * nc + c] = hist[j];
}

// Per chunk: wavefront w owns the chunk's keys [w * PER_WAVE, (w + 1) * PER_WAVE),
// read in blocks of 8 per lane with the next block's loads in flight.
// 1. Each tile's keys are counted per wavefront: the peers of each key's tile
//    among its step's lanes are found (a duplicate check in LDS, 12 ballots
//    when it finds one) and the first lane of each group adds the group's
//    size to the wavefront's count in LDS with one atomic; each key keeps its
//    tile and its rank among the wavefront's earlier keys of that tile.
// 2. A scan over the tiles of the chunk's totals gives each tile's start in
//    the chunk sorted by tile; the counts become per-(wavefront, tile) starts.
// 3. Each key's position l in the chunk sorted by tile (stable: equal tiles
//    keep the input order) is its (wavefront, tile) start plus its rank;
//    l -> input position goes to LDS.
// 4. Sorted position l is then written by thread l mod 256: the key (read
//    back, from L2) goes to the scanned matrix entry of its (tile, chunk)
//    plus l minus the tile's start in the chunk, so that each tile's run of
//    the chunk is written by consecutive lanes to consecutive addresses.
// Chunk 0 of each view writes the view's tile ranges.
__global__ __launch_bounds__(kTsThreads) void k_ts_scatter(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out,
                                                           const uint32_t* __restrict__ table,
                                                           const uint32_t* __restrict__ tstable, int n_views,
                                                           TsGeom tg, const uint32_t* __restrict__ tsm,
                                                           uint32_t* __restrict__ ranges) {
    constexpr int NW = kTsThreads / kWave;
    constexpr int PER_WAVE = kTsChunk / NW;
    constexpr int ITEMS = PER_WAVE / kWave;
    constexpr int PRE = kTsBins / kTsThreads;    // tiles per thread (contiguous)
    constexpr int KB = 8;                        // keys per lane per block
    static_assert(ITEMS == kTsItems && ITEMS % KB == 0, "items per lane");
    static_assert(kTsChunk <= 65536, "16-bit chunk positions");
    // per-(wavefront, tile) counts, then starts; after the ranking, the
    // destination of each tile's run minus its start in the chunk (uint32)
    __shared__ uint16_t cnt[NW][kTsBins];
    static_assert(sizeof(cnt) >= sizeof(uint32_t) * kTsBins, "run destinations fit over the counts");
    uint32_t* bml = reinterpret_cast<uint32_t*>(&cnt[0][0]);
    __shared__ uint16_t perm[kTsChunk];          // sorted position -> input position
    __shared__ uint8_t s_own[NW][kTsBins];       // per wavefront: a lane that holds the tile
    __shared__ uint32_t s_nop[kTsThreads];       // target of the non-leading lanes' atomics
    __shared__ uint64_t s_scan[NW];
    int v;
    uint32_t c;
    if (!ts_chunk_of(tstable, n_views, blockIdx.x, &v, &c)) return;
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const int nt = tg.ntiles[v], D = tg.depth_bits[v];
    const uint32_t nc = tstable[4 * v + 1], mb = tstable[4 * v + 2];
    const uint32_t seg_b = table[4 * v], seg_e = table[4 * v + 1];
    const uint32_t cstart = seg_b + c * kTsChunk;
    const int n_here = (int)min((uint32_t)kTsChunk, seg_e - cstart);
    // this thread's tiles [t * PRE, (t + 1) * PRE): their matrix entries (loads
    // unconditional, indices clamped into range, all in flight at once)
    uint32_t pre[PRE];
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
        const int j = min(t * PRE + q, nt - 1);
        pre[q] = tsm[mb + (uint32_t)j * nc + c];
    }
#pragma unroll
    for (int q = 0; q < PRE; ++q) {
#pragma unroll
        for (int r = 0; r < NW; ++r) cnt[r][t * PRE + q] = 0;
    }
    const int wbeg = w * PER_WAVE;
    const int nv = max(0, min(PER_WAVE, n_here - wbeg));      // keys of this wavefront
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // (a wavefront without keys reads the chunk's first key, which exists)
    const uint32_t last = nv > 0 ? cstart + (uint32_t)(wbeg + nv - 1) : cstart;
    auto load_block = [&](int i0, uint32_t (&dst)[KB]) {
#pragma unroll
        for (int u = 0; u < KB; ++u)
            dst[u] = keys_in[nv > 0 ? min(cstart + (uint32_t)(wbeg + (i0 + u) * kWave + lane), last) : last];
    };
    // peers of this lane's tile among the valid lanes.  Usually the 64 keys
    // of a step hold 64 different tiles (consecutive keys in depth order are
    // a few Gaussians' tile sets): every lane writes its id at its tile and
    // reads it back, and if no valid lane finds another's id, each lane is
    // its own only peer; otherwise 12 ballots find the peers.  The writes and
    // reads of a block of steps are issued back to back (a step's read may
    // also see a later step's write: that can only make a step take the
    // ballots, never hide a duplicate, since two lanes reading one byte read
    // one value).  Relaxed atomic LDS accesses: the read must see the other
    // lanes' writes, not the compiler's copy of its own.
    uint8_t* own = s_own[w];
    auto peers_of = [&](uint32_t tile, bool valid) -> uint64_t {
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 12; ++bit) {
            const bool set = (tile >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        return peers;
    };
    __syncthreads();
    // 1. counts per (wavefront, tile), and each key's tile and rank among the
    // wavefront's earlier keys of that tile, kept in registers for step 3.
    // The first lane of each tile's group takes the count and advances it in
    // one LDS atomic on the 32-bit word holding it (the neighbouring count in
    // the other half does not change: counts stay below 2^16); the other
    // lanes add 0 to a slot of their own, so the atomic needs no branch and
    // the compiler waits for the results only where they are used.  A
    // wavefront's LDS operations complete in issue order, so each group's
    // base counts every earlier key of its tile.
    uint32_t tr[ITEMS];                          // tile << 16 | rank
    uint32_t raw[ITEMS];                         // the word the group's first lane read
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) tr[i] = raw[i] = 0u;
    {
        uint32_t* wc = reinterpret_cast<uint32_t*>(&cnt[w][0]);
        uint32_t kc[KB], kn[KB];
        load_block(0, kn);
#pragma unroll
        for (int i0 = 0; i0 < ITEMS; i0 += KB) {
            if (i0 * kWave >= nv) break;
#pragma unroll
            for (int u = 0; u < KB; ++u) kc[u] = kn[u];
            if (i0 + KB < ITEMS) load_block(i0 + KB, kn);
            uint64_t pm[KB];
            uint32_t seen[KB];
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                kc[u] = (uint32_t)min((int)(kc[u] >> D), nt - 1);
                __hip_atomic_store(own + kc[u], (uint8_t)lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                seen[u] = __hip_atomic_load(own + kc[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const bool valid = (i0 + u) * kWave + lane < nv;
                if (__ballot(valid && seen[u] != (uint32_t)lane) == 0ull)
                    pm[u] = valid ? (uint64_t)1 << lane : 0ull;
                else
                    pm[u] = peers_of(kc[u], valid);
            }
#pragma unroll
            for (int u = 0; u < KB; ++u) {
                const uint32_t tile = kc[u];
                const uint64_t before = pm[u] & lt;
                const bool first = pm[u] != 0ull && before == 0ull;
                raw[i0 + u] = atomicAdd(first ? wc + (tile >> 1) : &s_nop[t],
                                        first ? (uint32_t)__popcll(pm[u]) << ((tile & 1u) * 16u) : 0u);
                // (tile, rank in the group, the group's first lane)
                tr[i0 + u] = (tile << 16) | ((uint32_t)__popcll(before) << 6) |
                             (pm[u] != 0ull ? (uint32_t)__builtin_ctzll(pm[u]) : 0u);
            }
        }
    }
    // every key's rank: its group's base, from the group's first lane
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t x = tr[i], tile = x >> 16;
        const uint32_t word = (uint32_t)__shfl((int)raw[i], (int)(x & 0x3Fu));
        tr[i] = (tile << 16) | (((word >> ((tile & 1u) * 16u)) & 0xFFFFu) + ((x >> 6) & 0x3Fu));
    }
    __syncthreads();
    // 2. tile starts within the chunk (scan over tiles), per-(wavefront, tile) starts
    uint32_t dstm[PRE];
    {
        uint32_t tot[PRE];
        uint32_t sum = 0;
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            uint32_t x = 0;
#pragma unroll
            for (int r = 0; r < NW; ++r) x += cnt[r][t * PRE + q];
            tot[q] = x;
            sum += x;
        }
        uint64_t all;
        uint32_t run = (uint32_t)(block_scan_u64(sum, s_scan, &all) - sum);
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int j = t * PRE + q;
            dstm[q] = pre[q] - run;
            uint32_t wr = run;
#pragma unroll
            for (int r = 0; r < NW; ++r) {
                const uint32_t x = cnt[r][j];
                cnt[r][j] = (uint16_t)wr;
                wr += x;
            }
            run += tot[q];
        }
    }
    __syncthreads();
    // 3. sorted position of every key: its (wavefront, tile) start plus its
    // rank from step 1 (no ballots, no dependence between keys)
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int r = i * kWave + lane;
        if (r < nv) perm[cnt[w][tr[i] >> 16] + (tr[i] & 0xFFFFu)] = (uint16_t)(wbeg + r);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PRE; ++q) bml[t * PRE + q] = dstm[q];
    __syncthreads();
    // 4. coalesced runs, KB sorted positions per lane at a time (reads of
    // positions past the chunk's keys are clamped and not written)
    for (int l0 = 0; l0 < n_here; l0 += KB * kTsThreads) {
        uint32_t src[KB], key[KB], val[KB];
#pragma unroll
        for (int u = 0; u < KB; ++u) src[u] = cstart + perm[min(l0 + u * kTsThreads + t, n_here - 1)];
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            key[u] = keys_in[src[u]];
            val[u] = vals_in[src[u]];
        }
#pragma unroll
        for (int u = 0; u < KB; ++u) {
            const int l = l0 + u * kTsThreads + t;
            if (l < n_here) {
                const uint32_t dst = bml[min((int)(key[u] >> D), nt - 1)] + (uint32_t)l;
                keys_out[dst] = key[u];
                vals_out[dst] = val[u];
            }
        }
    }
    if (c == 0) {
        uint2* R = reinterpret_cast<uint2*>(ranges) + tg.tile_base[v];
#pragma unroll
        for (int q = 0; q < PRE; ++q) {
            const int j = t * PRE + q;
            if (j < nt) {
                const uint32_t e0 = j + 1 < nt ? tsm[mb + (uint32_t)(j + 1) * nc] : seg_e;
                R[j] = make_uint2(pre[q], e0);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// driver
// ---------------------------------------------------------------------------

int launch_bin_sort(const gs_splats& sp, int64_t n, const gs_layout& L, const gs_bins& b, void* ws,
                    size_t ws_bytes, const gs_side_stream* side, hipStream_t s) {
    Workspace W;
    const size_t need = carve(n, L, b.capacity, (char*)ws, &W);
    if (ws_bytes < need) {
        set_error("bin_sort: workspace of %zu bytes, %zu needed", ws_bytes, need);
        return GS_ERR_WORKSPACE;
    }
    const int V = L.n_views;
    const int64_t m = (int64_t)V * n;
    // With many intersections per (view, Gaussian) the keys are emitted in
    // depth order (a sort of the (view, Gaussian)s by their depth bits) and
    // then sorted by their tile bits only; with few, the depth sort costs more
    // than the two passes it saves, and all 32 bits are sorted directly.  Both
    // give the same order: (tile, depth bits, Gaussian id).
    const bool depth_first = m > 0 && b.capacity >= kDepthFirstRatio * m;
    // (An LSD sort may split the key anywhere: the keys' bits below
    // split = min(kDepthSplit, D) are depth bits, the same for all of a
    // Gaussian's keys, so they are sorted per (view, Gaussian); the keys'
    // bits from split up are then sorted stably.)
    // With every view at most kTsBins tiles, the depth order takes all depth
    // bits and one stable partition by tile finishes (the single-pass tile
    // scatter); otherwise the depth order takes the low kDepthSplit bits and
    // radix passes sort the rest.
    const bool ts_path = depth_first && W.ts_len > 0;
    SortWs S = carve_sort(W.sort_words, V, W.max_chunks);
    int high_bits = 1, low_bits = 1;
    int splits[GS_MAX_VIEWS];
    for (int v = 0; v < V; ++v) {
        const int split = ts_path ? L.depth_bits[v] : std::min(kDepthSplit, L.depth_bits[v]);
        splits[v] = split;
        S.shift0[v] = depth_first ? split : 0;
        high_bits = std::max(high_bits, 32 - split);
        low_bits = std::max(low_bits, split);
    }
    S.passes = depth_first ? std::min(kPasses, (high_bits + 7) / 8) : kPasses;
    // depth sort: the low bits of each (view, Gaussian)'s keys
    SortWs SD = carve_sort(W.dsort_words, V, W.max_dchunks);
    SD.passes = std::min(kPasses, (low_bits + 7) / 8);
    int rc;
    EmitGeom eg;
    RangeGeom rg;
    memset(&eg, 0, sizeof(eg));
    TsGeom tg;
    memset(&tg, 0, sizeof(tg));
    for (int v = 0; v < GS_MAX_VIEWS; ++v) {
        eg.tiles_x[v] = v < V ? L.tiles_x[v] : 0;
        eg.tiles_y[v] = v < V ? L.tiles_y[v] : 0;
        eg.depth_bits[v] = v < V ? L.depth_bits[v] : 0;
        eg.split[v] = v < V ? splits[v] : 0;
        rg.depth_bits[v] = eg.depth_bits[v];
        rg.tiles_x[v] = eg.tiles_x[v];
        tg.ntiles[v] = v < V ? L.tile_base[v + 1] - L.tile_base[v] : 0;
        tg.depth_bits[v] = eg.depth_bits[v];
    }
    for (int v = 0; v <= GS_MAX_VIEWS; ++v) tg.tile_base[v] = v <= V ? L.tile_base[v] : L.tile_base[V];
    eg.tile = L.tile;
    eg.cull = L.cull;
    for (int v = 0; v <= GS_MAX_VIEWS; ++v) rg.tile_base[v] = v <= V ? L.tile_base[v] : L.tile_base[V];
    const float4* rec = reinterpret_cast<const float4*>(sp.rec);
    uint4* rows = reinterpret_cast<uint4*>(b.rows);
    const unsigned gm = (unsigned)std::max<int64_t>((m + 255) / 256, 1);
    // status cleared, tile rows and depth keys per (view, Gaussian)
    hipLaunchKernelGGL(k_row_count, dim3(gm), dim3(256), 0, s, rec, sp.tiles, n, m, eg, W.row_count, b.status,
                       W.dkey, W.dval, W.dtable, SD.dcount, V, depth_first);
    if ((rc = check_launch("row_count")) != GS_OK) return rc;
    // the caller's side stream, if any, takes the depth order
    const bool forked = depth_first && side != nullptr;
    const hipStream_t ds = forked ? (hipStream_t)side->stream : s;
    if (forked) {
        if (hipEventRecord((hipEvent_t)side->fork, s) != hipSuccess ||
            hipStreamWaitEvent(ds, (hipEvent_t)side->fork, 0) != hipSuccess) {
            set_error("bin_sort: cannot fork to the side stream");
            return GS_ERR_HIP;
        }
    }
    if (depth_first) {
        // depth order: a stable sort of the (view, Gaussian)s by depth bits,
        // then the scan of their tile counts in that order (each one's first
        // position); independent of the scans and row slots below
        if ((rc = radix_sort_views<kDepthItems>(W.dkey, W.dval, W.dkey_tmp, W.dval_tmp, W.dtable, V, SD, b.status,
                                                ds)) != GS_OK)
            return rc;
        const uint32_t* perm = SD.passes % 2 == 0 ? W.dval : W.dval_tmp;
        if ((rc = scan_exclusive(sp.tiles, m, W.dpos, W.dblock_sums, nullptr, ds, perm)) != GS_OK) return rc;
    }
    if (forked && hipEventRecord((hipEvent_t)side->join, ds) != hipSuccess) {
        set_error("bin_sort: cannot join the side stream");
        return GS_ERR_HIP;
    }
    // offsets and row offsets, the view table, the row slots
    if ((rc = scan_exclusive(sp.tiles, m, b.offsets, W.block_sums, b.status, s)) != GS_OK) return rc;
    hipLaunchKernelGGL(k_view_table, dim3(1), dim3(256), 0, s, b.offsets, n, V, b.capacity, W.table,
                       b.status, S.dcount, ts_path ? W.tstable : nullptr, tg);
    if ((rc = check_launch("view_table")) != GS_OK) return rc;
    if ((rc = scan_exclusive(W.row_count, m, b.row_offsets, W.block_sums, nullptr, s)) != GS_OK) return rc;
    if (m > 0) {
        hipLaunchKernelGGL(k_rows, dim3(gm), dim3(256), 0, s, rec, sp.tiles, b.offsets, b.row_offsets, n, m,
                           eg, b.row_capacity, rows, b.status);
        if ((rc = check_launch("rows")) != GS_OK) return rc;
    }
    if (forked && hipStreamWaitEvent(s, (hipEvent_t)side->join, 0) != hipSuccess) {
        set_error("bin_sort: cannot wait for the side stream");
        return GS_ERR_HIP;
    }
    // keys (in depth order if depth_first), then the sort; the emit goes to
    // the buffer that leaves the sorted keys in bins.keys
    uint32_t* ek = (ts_path || S.passes % 2 != 0) ? W.keys_tmp : b.keys;
    uint32_t* ev = (ts_path || S.passes % 2 != 0) ? W.vals_tmp : b.vals;
    uint32_t* ok = S.passes % 2 == 0 ? W.keys_tmp : b.keys;
    uint32_t* ov = S.passes % 2 == 0 ? W.vals_tmp : b.vals;
    if (m > 0 && b.row_capacity > 0) {
        hipLaunchKernelGGL(k_emit, dim3((unsigned)((b.row_capacity + kEmitG - 1) / kEmitG)), dim3(kEmitG), 0, s,
                           rec, rows, b.row_offsets, b.offsets, depth_first ? W.dpos : nullptr, n, m, eg,
                           b.capacity, b.row_capacity, ek, ev);
        if ((rc = check_launch("emit_keys")) != GS_OK) return rc;
    }
    if (ts_path) {
        // a multiple of 8 workgroups covers every chunk under the XCD dealing
        const unsigned tgrid = (unsigned)((W.max_ts_chunks + 7) / 8 * 8);
        hipLaunchKernelGGL(k_ts_count, dim3(tgrid), dim3(kTsThreads), 0, s, ek, W.table, W.tstable, V, tg, W.tsm,
                           b.ranges);
        if ((rc = check_launch("ts_count")) != GS_OK) return rc;
        if ((rc = scan_exclusive(W.tsm, W.ts_len, W.tsm, W.ts_sums, nullptr, s)) != GS_OK) return rc;
        hipLaunchKernelGGL(k_ts_scatter, dim3(tgrid), dim3(kTsThreads), 0, s, ek, ev, b.keys, b.vals, W.table,
                           W.tstable, V, tg, W.tsm, b.ranges);
        return check_launch("ts_scatter");
    }
    if ((rc = radix_sort_views<kSortItems>(ek, ev, ok, ov, W.table, V, S, b.status, s)) != GS_OK) return rc;
    const int64_t nt = L.tile_base[V];
    const int64_t rgrid =
        std::max<int64_t>(1, std::min<int64_t>((std::max(b.capacity / 4, nt) + 255) / 256, kRangeBlocks));
    hipLaunchKernelGGL(k_ranges, dim3((unsigned)rgrid), dim3(256), 0, s, b.keys, W.table, V, rg, b.ranges);
    return check_launch("ranges");
}

}  // namespace gs
