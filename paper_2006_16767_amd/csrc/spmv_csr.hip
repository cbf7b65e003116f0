// Row-major kernels (Section 4.1): SpMV, and SpMSpV with value validation
// against a bitvector of supp(x) (Section 6.1). Both with the two workload
// distributions of Section 4.2.1:
//
//  * direct   - a fixed group of L lanes per row (L = 1 is the classic
//               thread-per-row kernel; L = 64 a whole wave per row). The
//               group strides through the row, each lane keeps a partial sum
//               and the group reduces with cross-lane shuffles.
//  * balanced - merge-path tiles: the merge of row ends and nonzeros is cut
//               into equal pieces of kTile items, so every workgroup gets
//               the same amount of (rows + nonzeros) whatever the row-length
//               distribution. A tile stages its products in LDS with
//               coalesced loads; each thread then walks kIpt merge items,
//               partial sums that cross thread boundaries are combined with a
//               segmented scan, and a row that spans tiles is finished by a
//               small fix-up pass in tile order (deterministic).
//
// With validation (the CSR SpMSpV pattern) a product is formed only where
// bit(col) is set; x values are read from the scattered copy xd, so neither
// vals[k] nor xd[col] is touched for ineffective entries. For BOOL the
// product is the bit itself.
#include <algorithm>

#include "common.hpp"
#include "csr_tile.hpp"
#include "internal.hpp"

namespace spx {

// --------------------------------------------------------------- direct
template <int DT, int L, bool VALID>
__global__ __launch_bounds__(kBlock) void k_csr_direct(int32_t m, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       const typename SR<DT>::V* __restrict__ vals,
                                                       const typename SR<DT>::X* __restrict__ x,
                                                       const uint32_t* __restrict__ bits,
                                                       typename SR<DT>::Y* __restrict__ y) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    constexpr int kRowsPerBlock = kBlock / L;
    const int64_t row = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / L;
    const int g = threadIdx.x % L;
    if (row >= m) return;  // whole groups leave together (L divides 64)
    const int k0 = row_ptr[row], k1 = row_ptr[row + 1];
    // eight loads in flight per lane, predicated on the row's end: a short
    // row (up to 8 * L entries) costs one round trip; each load slot keeps
    // its own partial sum (bounded chains on hub rows)
    ChunkedAcc<DT, 8> acc;
    for (int k = k0 + g; k < k1; k += 8 * L) {
        int c[8];
        bool on[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            on[u] = k + u * L < k1;
            c[u] = on[u] ? col_idx[k + u * L] : 0;
        }
        if constexpr (VALID) {
#pragma unroll
            for (int u = 0; u < 8; ++u) on[u] = on[u] && test_bit(bits, c[u]);
        }
        typename S::V a[8];
        typename S::X b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            a[u] = on[u] ? S::val(vals, k + u * L) : (typename S::V)0;
            b[u] = on[u] ? S::xval(x, c[u]) : (typename S::X)0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (on[u]) acc.part[u] = S::fma(a[u], b[u], acc.part[u]);
        acc.end_round();
    }
    const Acc sum = group_reduce<DT, L>(acc.total());
    if (g == 0) y[row] = S::out(sum);
}

// --------------------------------------------------------------- balanced
// Merge-path partition: boundary b of tile size T sits at merge diagonal
// d = min(b * T, m + nnz); part[2b] = rows finished before d, part[2b+1] =
// nonzeros consumed before d. Depends on the matrix only, so a handle
// computes it once.
__global__ __launch_bounds__(kBlock) void k_merge_partition(int32_t m, int32_t nnz,
                                                            const int32_t* __restrict__ row_ptr, int64_t tiles,
                                                            int32_t tile, int32_t* __restrict__ part) {
    const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (b > tiles) return;
    const int64_t d = std::min<int64_t>(b * tile, (int64_t)m + nnz);
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)row_ptr[mid + 1] + mid >= d)
            hi = mid;
        else
            lo = mid + 1;
    }
    part[2 * b] = lo;
    part[2 * b + 1] = (int)(d - lo);
}

template <int DT, bool VALID, int TILE>
__global__ __launch_bounds__(kBlock) void k_csr_merge(int32_t m, const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col_idx,
                                                      const typename SR<DT>::V* __restrict__ vals,
                                                      const typename SR<DT>::X* __restrict__ x,
                                                      const uint32_t* __restrict__ bits,
                                                      typename SR<DT>::Y* __restrict__ y,
                                                      const int32_t* __restrict__ part, int64_t tiles,
                                                      int32_t* __restrict__ carry_row,
                                                      typename SR<DT>::Acc* __restrict__ carry_val) {
    __shared__ CsrTileLds<DT, TILE> L;
    csr_merge_tile<DT, VALID, TILE>(xcd_tile(blockIdx.x, tiles), m, row_ptr, col_idx, vals, x, bits, y, part,
                                    carry_row, carry_val, L);
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_csr_merge_fixup(int32_t tiles,
                                                            const int32_t* __restrict__ carry_row,
                                                            const typename SR<DT>::Acc* __restrict__ carry_val,
                                                            typename SR<DT>::Y* __restrict__ y, Unscatter un) {
    using X = typename SR<DT>::X;
    const int64_t first = (int64_t)blockIdx.x * kBlock + threadIdx.x, stride = (int64_t)gridDim.x * kBlock;
    csr_merge_fixup_range<DT>(first, stride, tiles, carry_row, carry_val, y);
    // the scattered x back to zero (the product that read it has finished):
    // entry by entry for a sparse x (several entries of one bitvector word
    // store the same 0), the whole buffers with coalesced stores once x
    // holds more than n / 16 entries (fewer bytes than the scattered lines)
    X z = (X)0;
    if constexpr (DT == SPX_F32_MINPLUS) z = __builtin_inff();
    if ((int64_t)un.nnz_x * 16 > un.n) {
        if (un.bits)
            for (int64_t w = first; w < ((int64_t)un.n + 31) / 32; w += stride) un.bits[w] = 0u;
        if (un.xd)
            for (int64_t j = first; j < un.n; j += stride) ((X*)un.xd)[j] = z;
        return;
    }
    for (int64_t e = first; e < un.nnz_x; e += stride) {
        const int32_t j = un.map ? un.map[un.idx[e]] : un.idx[e];
        if (un.bits) un.bits[j >> 5] = 0u;
        if (un.xd) ((X*)un.xd)[j] = z;
    }
}


// Balanced SpMV / bitvector SpMSpV over the column-sorted copy (2048-item
// tiles).
template <int DT, bool VALID>
__global__ __launch_bounds__(kBlock) void k_csr_merge_sorted(int32_t m, const int32_t* __restrict__ row_ptr,
                                                             const uint32_t* __restrict__ pk,
                                                             const typename SR<DT>::V* __restrict__ vals,
                                                             const typename SR<DT>::X* __restrict__ x,
                                                             const uint32_t* __restrict__ bits,
                                                             typename SR<DT>::Y* __restrict__ y,
                                                             const int32_t* __restrict__ part, int64_t tiles,
                                                             int32_t* __restrict__ carry_row,
                                                             typename SR<DT>::Acc* __restrict__ carry_val) {
    constexpr int kTile = 2048;
    __shared__ CsrTileLds<DT, kTile> L;
    csr_merge_tile_core<DT, kTile, kBlock>(xcd_tile(blockIdx.x, tiles), m, row_ptr, y, part, carry_row, carry_val, L,
                                           [&](int k0, int Q, typename SR<DT>::Acc* prod) {
                                               csr_stage_sorted<DT, VALID, kTile / kBlock, kBlock>(k0, Q, pk, vals,
                                                                                                   x, bits, prod);
                                           });
}

// --------------------------------------------------------------- LDS bitvector
// Row-major SpMSpV with the bitvector of supp(x) held in LDS. One persistent
// 1024-thread workgroup per CU copies the bitvector (n / 8 bytes, up to
// kLdsBitsMax) into LDS once, then takes merge tiles in XCD-contiguous
// order. The per-entry validation becomes an LDS read; only effective
// entries touch vals and the scattered x values.
constexpr int kBitThreads = 1024;
constexpr int kBitTile = 2048;
constexpr int kLdsTotal = 160 * 1024;  // LDS per workgroup on gfx950

template <int DT>
__global__ __launch_bounds__(kBitThreads) void k_csr_bitlds(int32_t m, int32_t n, const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col_idx,
                                                            const typename SR<DT>::V* __restrict__ vals,
                                                            const typename SR<DT>::X* __restrict__ x,
                                                            const uint32_t* __restrict__ bits,
                                                            typename SR<DT>::Y* __restrict__ y,
                                                            const int32_t* __restrict__ part, int64_t tiles,
                                                            int32_t* __restrict__ carry_row,
                                                            typename SR<DT>::Acc* __restrict__ carry_val) {
    extern __shared__ __align__(16) uint32_t s_bits[];
    __shared__ CsrTileLds<DT, kBitTile> L;
    const int nwords = (n + 31) >> 5;
    for (int w = threadIdx.x; w < nwords; w += kBitThreads) s_bits[w] = bits[w];
    __syncthreads();
    // XCD-contiguous order over the persistent grid
    for (int64_t bt = blockIdx.x; bt < tiles; bt += gridDim.x)
        csr_merge_tile_nt<DT, true, kBitTile, kBitThreads>(
            xcd_tile(bt, tiles), m, row_ptr, col_idx, vals, [x](int c) { return SR<DT>::xval(x, c); }, s_bits, y,
            part, carry_row, carry_val, L);
}

// static LDS of k_csr_bitlds plus the bitvector must fit one CU's LDS
static size_t bitlds_static(int dtype) {
    // every semiring's accumulator is at most 4 bytes except FP64's
    return (dtype == SPX_F64 ? sizeof(CsrTileLds<SPX_F64, kBitTile>) : sizeof(CsrTileLds<SPX_F32, kBitTile>)) + 64;
}
bool bitlds_fits(int32_t n, int dtype) {
    return (size_t)((n + 31) / 32) * 4 + bitlds_static(dtype) + 512 <= (size_t)kLdsTotal;
}

// --------------------------------------------------------------- launch
// Lanes per row of the direct distribution: the largest power of two up to
// half the average row length, at most 32 (measured on MI355X over uniform
// rows of 7 to 205 entries: 2, 8, 16, 32 and 32 lanes were fastest at
// averages 7, 16, 32, 64 and 205).
static int pick_lanes(int32_t m, int32_t nnz) {
    const double avg = m > 0 ? (double)nnz / m : 0.0;
    int L = 1;
    while (L < 32 && 4.0 * L <= avg) L <<= 1;
    return L;
}

static int merge_tile(const spx_plan* plan) { return plan->tile == 4096 ? 4096 : 2048; }
// plan->tile = 1 asks the balanced row-major SpMSpV to keep the bitvector in
// LDS (persistent workgroups, when n / 8 bytes fit next to the tile).
static bool want_bitlds(const spx_plan* plan, int32_t n, int dtype) {
    return plan->pattern == SPX_PAT_CSR_SPMSPV && plan->distribution == SPX_DIST_BALANCED && plan->tile == 1 &&
           bitlds_fits(n, dtype);
}

size_t spmv_csr_ws(int32_t m, int32_t nnz, const spx_plan* plan) {
    if (!plan || plan->distribution != SPX_DIST_BALANCED) return 0;
    const int64_t tiles = ceil_div((int64_t)m + nnz, merge_tile(plan));
    Sizer z;
    z.take<int32_t>(2 * (tiles + 1));
    z.take<int32_t>(tiles);
    z.take<double>(tiles);
    return z.used;
}

spx_status merge_partition(int32_t m, int32_t nnz, const int32_t* row_ptr, int tile, int32_t* part, hipStream_t s) {
    const int64_t tiles = ceil_div((int64_t)m + nnz, tile);
    k_merge_partition<<<(unsigned)ceil_div(tiles + 1, kBlock), kBlock, 0, s>>>(m, nnz, row_ptr, tiles, tile, part);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

template <int DT, bool VALID>
static spx_status launch_csr_t(const spx_csr* A, const void* x, const uint32_t* bits, void* y,
                               const spx_plan* plan, const int32_t* part, Arena& ws, hipStream_t s,
                               const Unscatter* un, bool* cleared, const TileSorted* ts) {
    using S = SR<DT>;
    const auto* vals = (const typename S::V*)A->vals;
    const auto* xv = (const typename S::X*)x;
    auto* yv = (typename S::Y*)y;
    if (A->m == 0) return SPX_OK;
    if (plan->distribution == SPX_DIST_DIRECT) {
        int L = plan->lanes > 0 ? plan->lanes : pick_lanes(A->m, A->nnz);
        const int64_t blocks = ceil_div(A->m, kBlock / L);
        switch (L) {
#define SPX_L(LL)                                                                                   \
    case LL:                                                                                        \
        k_csr_direct<DT, LL, VALID><<<(unsigned)blocks, kBlock, 0, s>>>(A->m, A->row_ptr,           \
                                                                        A->col_idx, vals, xv, bits, yv); \
        break;
            SPX_L(1)
            SPX_L(2)
            SPX_L(4)
            SPX_L(8)
            SPX_L(16)
            SPX_L(32)
            SPX_L(64)
#undef SPX_L
            default:
                return fail(SPX_ERR_ARG, "lanes must be a power of two in [1, 64]");
        }
        SPX_HIP(hipGetLastError());
        return SPX_OK;
    }
    if (plan->distribution == SPX_DIST_BALANCED) {
        const int T = merge_tile(plan);
        const int64_t tiles = ceil_div((int64_t)A->m + A->nnz, T);
        int32_t* own_part = ws.take<int32_t>(2 * (tiles + 1));
        int32_t* crow = ws.take<int32_t>(tiles);
        auto* cval = ws.take<typename S::Acc>(tiles);
        if (!own_part || !crow || !cval) return fail(SPX_ERR_WORKSPACE, "spmv balanced: workspace too small");
        if (!part) {
            SPX_TRY(merge_partition(A->m, A->nnz, A->row_ptr, T, own_part, s));
            part = own_part;
        }
        if (VALID && want_bitlds(plan, A->n, DT)) {
            int dev = 0, cus = 256;
            SPX_HIP(hipGetDevice(&dev));
            SPX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            const int grid = (int)std::min<int64_t>(tiles, std::max(1, cus));
            const size_t lds = (size_t)((A->n + 31) / 32) * 4;
            SPX_HIP(hipFuncSetAttribute((const void*)k_csr_bitlds<DT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds));
            k_csr_bitlds<DT><<<grid, kBitThreads, lds, s>>>(A->m, A->n, A->row_ptr, A->col_idx, vals, xv, bits, yv,
                                                           part, tiles, crow, cval);
        } else if (ts && ts->pk && T == 2048) {
            k_csr_merge_sorted<DT, VALID><<<(unsigned)tiles, kBlock, 0, s>>>(
                A->m, A->row_ptr, ts->pk, (const typename S::V*)ts->vals, xv, bits, yv, part, tiles, crow, cval);
        } else if (T == 4096)
            k_csr_merge<DT, VALID, 4096><<<(unsigned)tiles, kBlock, 0, s>>>(A->m, A->row_ptr, A->col_idx, vals, xv,
                                                                           bits, yv, part, tiles, crow, cval);
        else
            k_csr_merge<DT, VALID, 2048><<<(unsigned)tiles, kBlock, 0, s>>>(A->m, A->row_ptr, A->col_idx, vals, xv,
                                                                           bits, yv, part, tiles, crow, cval);
        SPX_HIP(hipGetLastError());
        const Unscatter u = un ? *un : Unscatter{};
        const int64_t work = std::max<int64_t>(tiles, (int64_t)u.nnz_x * 16 > u.n ? u.n : u.nnz_x);
        k_csr_merge_fixup<DT><<<(unsigned)std::min<int64_t>(ceil_div(work, kBlock), 8192), kBlock, 0, s>>>(
            (int32_t)tiles, crow, cval, yv, u);
        SPX_HIP(hipGetLastError());
        if (cleared) *cleared = un != nullptr;
        return SPX_OK;
    }
    return fail(SPX_ERR_ARG, "unknown distribution");
}

spx_status launch_spmv_csr(const spx_csr* A, const void* x, const uint32_t* bits, void* y,
                           const spx_plan* plan, const int32_t* part, Arena& ws, hipStream_t s,
                           const Unscatter* un, bool* cleared, const TileSorted* ts) {
    if (cleared) *cleared = false;
    const bool valid = plan->pattern == SPX_PAT_CSR_SPMSPV;
    switch (A->dtype) {
#define SPX_DT(DT)                                                                            \
    case DT:                                                                                  \
        return valid ? launch_csr_t<DT, true>(A, x, bits, y, plan, part, ws, s, un, cleared, ts)  \
                     : launch_csr_t<DT, false>(A, x, bits, y, plan, part, ws, s, un, cleared, ts);
        SPX_DT(SPX_F32)
        SPX_DT(SPX_F64)
        SPX_DT(SPX_I32)
        SPX_DT(SPX_BOOL)
        SPX_DT(SPX_F32_MINPLUS)
#undef SPX_DT
    }
    return fail(SPX_ERR_DTYPE, "spmv: unknown dtype");
}

// --------------------------------------------------------------- column-sorted copy
// tile_of[k] = the 2048-item tile holding entry k (a workgroup per tile)
__global__ __launch_bounds__(kBlock) void k_ts_tile_of(const int32_t* __restrict__ part, int64_t tiles,
                                                       int32_t* __restrict__ tile_of) {
    const int64_t t = blockIdx.x;
    if (t >= tiles) return;
    const int k0 = part[2 * t + 1], k1 = part[2 * t + 3];
    for (int k = k0 + (int)threadIdx.x; k < k1; k += kBlock) tile_of[k] = (int32_t)t;
}

// keys = column, vals = position (the first sort: by column)
__global__ __launch_bounds__(kBlock) void k_ts_pairs(int64_t nnz, const int32_t* __restrict__ col,
                                                     uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += stride) {
        keys[k] = (uint32_t)col[k];
        vals[k] = (uint32_t)k;
    }
}

// keys = tile of each position (the second, stable sort: by tile)
__global__ __launch_bounds__(kBlock) void k_ts_tile_keys(int64_t nnz, const uint32_t* __restrict__ pos,
                                                         const int32_t* __restrict__ tile_of,
                                                         uint32_t* __restrict__ keys) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nnz; k += stride)
        keys[k] = (uint32_t)tile_of[pos[k]];
}

// Sorted position p holds entry src = pos[p], of the same tile (the tiles'
// ranges are contiguous and the sort keeps their sizes): its word packs the
// column with src's slot in the tile.
__global__ __launch_bounds__(kBlock) void k_ts_fill(int64_t nnz, const uint32_t* __restrict__ pos,
                                                    const int32_t* __restrict__ tile_of,
                                                    const int32_t* __restrict__ part,
                                                    const int32_t* __restrict__ col,
                                                    const int32_t* __restrict__ src_of_A,
                                                    uint32_t* __restrict__ pk, int32_t* __restrict__ src) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < nnz; p += stride) {
        const uint32_t e = pos[p];
        const int32_t k0 = part[2 * tile_of[p] + 1];
        pk[p] = (uint32_t)col[e] | ((e - (uint32_t)k0) << kTsColBits);
        src[p] = src_of_A ? src_of_A[e] : (int32_t)e;
    }
}

void tile_sorted_free(TileSorted* ts) {
    void* ptrs[] = {ts->pk, ts->vals, ts->src};
    for (void* p : ptrs)
        if (p) hipFree(p);
    *ts = TileSorted{};
}

static int bits_for(int64_t n) {
    int b = 1;
    while (b < 31 && (int64_t(1) << b) < n) ++b;
    return b;
}

spx_status tile_sorted_build(const spx_csr& A, const int32_t* part, const int32_t* src_of_A, TileSorted* out,
                             hipStream_t s) {
    const int64_t nnz = A.nnz;
    if (A.n > (1 << kTsColBits)) return fail(SPX_ERR_UNSUPPORTED, "column-sorted copy: n above 2^21");
    if (nnz == 0 || A.m == 0) return SPX_OK;
    const int64_t tiles = ceil_div((int64_t)A.m + nnz, 2048);
    const int vs = value_size(A.dtype);
    TileSorted ts;
    uint32_t *keys = nullptr, *vals = nullptr, *keys2 = nullptr, *vals2 = nullptr;
    int32_t *rws = nullptr, *tile_of = nullptr;
    spx_status st = SPX_OK;
    do {
        if (hipMalloc((void**)&ts.pk, nnz * 4) != hipSuccess || hipMalloc((void**)&ts.src, nnz * 4) != hipSuccess ||
            (vs > 0 && hipMalloc(&ts.vals, nnz * vs) != hipSuccess) ||
            hipMalloc((void**)&keys, nnz * 4) != hipSuccess || hipMalloc((void**)&vals, nnz * 4) != hipSuccess ||
            hipMalloc((void**)&keys2, nnz * 4) != hipSuccess || hipMalloc((void**)&vals2, nnz * 4) != hipSuccess ||
            hipMalloc((void**)&tile_of, nnz * 4) != hipSuccess ||
            hipMalloc((void**)&rws, radix_ws_elems(nnz) * 4) != hipSuccess) {
            st = fail(SPX_ERR_ALLOC, "column-sorted copy: allocation failed");
            break;
        }
        const int grid = (int)std::min<int64_t>(ceil_div(nnz, kBlock), 8192);
        k_ts_tile_of<<<(unsigned)tiles, kBlock, 0, s>>>(part, tiles, tile_of);
        k_ts_pairs<<<grid, kBlock, 0, s>>>(nnz, A.col_idx, keys, vals);
        if (hipGetLastError() != hipSuccess) {
            st = fail(SPX_ERR_HIP, "column-sorted copy: kernels");
            break;
        }
        bool alt = false;
        if ((st = radix_sort_pairs(keys, vals, keys2, vals2, nnz, bits_for(A.n), rws, s, &alt))) break;
        uint32_t* pos = alt ? vals2 : vals;
        uint32_t* k2 = alt ? keys2 : keys;
        uint32_t* other_k = alt ? keys : keys2;
        uint32_t* other_v = alt ? vals : vals2;
        k_ts_tile_keys<<<grid, kBlock, 0, s>>>(nnz, pos, tile_of, k2);
        if (hipGetLastError() != hipSuccess) {
            st = fail(SPX_ERR_HIP, "column-sorted copy: kernels");
            break;
        }
        bool alt2 = false;
        if ((st = radix_sort_pairs(k2, pos, other_k, other_v, nnz, bits_for(tiles), rws, s, &alt2))) break;
        uint32_t* pos2 = alt2 ? other_v : pos;
        k_ts_fill<<<grid, kBlock, 0, s>>>(nnz, pos2, tile_of, part, A.col_idx, src_of_A, ts.pk, ts.src);
        if (hipGetLastError() != hipSuccess) {
            st = fail(SPX_ERR_HIP, "column-sorted copy: kernels");
            break;
        }
        if (vs > 0 && (st = gather_perm(A.vals, (const int32_t*)pos2, ts.vals, nnz, vs, s))) break;
        if (hipStreamSynchronize(s) != hipSuccess) st = fail(SPX_ERR_HIP, "column-sorted copy: sync");
    } while (0);
    for (void* p : {(void*)keys, (void*)vals, (void*)keys2, (void*)vals2, (void*)rws, (void*)tile_of})
        if (p) hipFree(p);
    if (st != SPX_OK) {
        tile_sorted_free(&ts);
        return st;
    }
    *out = ts;
    return SPX_OK;
}

}  // namespace spx
