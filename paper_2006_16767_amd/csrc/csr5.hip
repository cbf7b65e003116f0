// CSR5-style copy of A for the row-major SpMV: the fourth candidate of the
// storage-format pre-selection (the paper's extension, Section 8, names
// CSR5 among the formats an SMAT-style pre-selector picks from; the tiling
// follows Liu and Vinter's CSR5, ICS 2015, with the tile sized for a 64-lane
// wave and the empty rows handled by an ordinal map instead of per-tile
// offsets).
//
// Layout: the entries, in CSR order, are cut into tiles of kC5Tile = 64 x
// kC5Sigma. Lane l of a tile owns the kC5Sigma consecutive entries
// [l * sigma, (l + 1) * sigma) of the tile, stored transposed (the lane's
// entry j at j * 64 + l), so that every step of a wave reads 64 consecutive
// column indices and values. Per lane one word of row-start bits (bit j:
// the lane's entry j is the first entry of its row); per tile the ordinal,
// among the non-empty rows, of its first row start; nz_rows maps an ordinal
// to its row and empty_rows lists the rows with no entry, so empty rows
// need no correction inside a tile. The copy is built once from a host copy
// of row_ptr (bits and ordinals) and one transposing kernel.
//
// y = A x, two launches:
//  k_c5_spmv   one wave per tile. Each lane sums its entries in registers
//              (kC5Sigma in flight) and writes the rows that start and end
//              inside it. The sum before its first row start (head) and the
//              one after its last (tail) cross lanes: a backward segmented
//              scan over the heads gives, for the lane holding a row's start,
//              the heads of the following lanes up to and including the
//              next lane with a start; that row is then complete. The row
//              still open at the tile's end leaves its partial sum (trail),
//              and the part of the tile before its first start its lead.
//  k_c5_fixup  one wave per tile that holds a row start: the trail plus the
//              leads of the following tiles up to and including the next
//              tile with a start, 64 tiles a step, written to that row; and
//              the empty rows are zeroed.
// Every sum has a fixed order (in-lane, then a fixed scan tree, then tile
// order), so a call repeats its bits. The same tiles serve the bitvector
// SpMSpV (k_c5_spmspv_lds), with the bitvector of supp(x) held in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace spx {

constexpr int kC5Sigma = 16;
constexpr int kC5Tile = kWave * kC5Sigma;
static_assert(kC5Sigma <= 32, "one 32-bit word of row-start bits per lane");

template <typename T>
__device__ __forceinline__ T shfl_down(T v, int delta) {
    return __shfl_down(v, delta, kWave);
}

// CSR position of the copy's cell q (q = tile * kC5Tile + j * 64 + lane).
__device__ __forceinline__ int64_t c5_source(int64_t q) {
    const int64_t t = q / kC5Tile;
    const int r = (int)(q - t * kC5Tile);
    return t * kC5Tile + (int64_t)(r % kWave) * kC5Sigma + r / kWave;
}

__global__ __launch_bounds__(kBlock) void k_c5_cols(int64_t cells, int32_t nnz, const int32_t* __restrict__ col_idx,
                                                    int32_t* __restrict__ col) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < cells; q += stride) {
        const int64_t k = c5_source(q);
        col[q] = k < nnz ? col_idx[k] : 0;  // padding cells are never gathered
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_c5_vals(int64_t cells, int32_t nnz, const T* __restrict__ csr_vals,
                                                    T* __restrict__ vals) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < cells; q += stride) {
        const int64_t k = c5_source(q);
        vals[q] = k < nnz ? csr_vals[k] : (T)0;
    }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_c5_spmv(int64_t ntiles, int32_t nnz, const int32_t* __restrict__ col,
                                                    const typename SR<DT>::V* __restrict__ vals,
                                                    const uint32_t* __restrict__ flags,
                                                    const int32_t* __restrict__ tile_start,
                                                    const int32_t* __restrict__ nz_rows,
                                                    const typename SR<DT>::X* __restrict__ x,
                                                    typename SR<DT>::Y* __restrict__ y,
                                                    typename SR<DT>::Acc* __restrict__ lead,
                                                    typename SR<DT>::Acc* __restrict__ trail) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (t >= ntiles) return;  // uniform over the wave; no workgroup barrier below
    const int lane = lane_id();
    const int64_t base = t * kC5Tile;
    const int64_t first = base + (int64_t)lane * kC5Sigma;  // CSR position of the lane's entry 0
    const uint32_t fl = flags[t * kWave + lane];
    int c[kC5Sigma];
    typename S::V a[kC5Sigma];
    typename S::X b[kC5Sigma];
#pragma unroll
    for (int j = 0; j < kC5Sigma; ++j) c[j] = col[base + j * kWave + lane];
#pragma unroll
    for (int j = 0; j < kC5Sigma; ++j) a[j] = S::val(vals, base + j * kWave + lane);
#pragma unroll
    for (int j = 0; j < kC5Sigma; ++j) b[j] = first + j < nnz ? S::xval(x, c[j]) : (typename S::X)0;
    const int nfl = __popc(fl);
    int ord = tile_start[t] + wave_incl_scan(nfl) - nfl;  // ordinal of the lane's first row start
    Acc run = S::zero(), head = S::zero();
    bool seen = false;
#pragma unroll
    for (int j = 0; j < kC5Sigma; ++j) {
        if ((fl >> j) & 1u) {
            if (seen) {
                y[nz_rows[ord]] = S::out(run);  // a row that starts and ends in this lane
                ++ord;
            } else {
                head = run;
                seen = true;
            }
            run = S::zero();
        }
        if (first + j < nnz) run = S::fma(a[j], b[j], run);
    }
    if (!seen) head = run;
    // Backward segmented scan: v = the heads of lanes [lane, next lane with a
    // start], that lane included; f = whether such a lane was met.
    Acc v = head;
    int f = seen ? 1 : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const Acc vo = shfl_down(v, d);
        const int fo = shfl_down(f, d);
        if (lane + d < kWave && !f) {
            v = S::add(v, vo);
            f = fo;
        }
    }
    const Acc vn = shfl_down(v, 1);
    const int fn = shfl_down(f, 1);
    if (seen) {
        // the lane's last row: its tail plus the heads up to the next start
        const Acc tot = lane + 1 < kWave ? S::add(run, vn) : run;
        if (lane + 1 < kWave && fn)
            y[nz_rows[ord]] = S::out(tot);
        else
            trail[t] = tot;  // the tile's last start: the row is still open
    }
    if (lane == 0) lead[t] = v;
}

// ------------------------------------------------------------------ bitvector SpMSpV
// The bitvector SpMSpV over the same tiles, with the bitvector of supp(x) in
// LDS: one persistent 1024-thread workgroup per CU copies it (n / 8 bytes, at
// most kC5LdsWords words) once; then each of its 16 waves walks its own tiles
// (no barrier), and while it sums tile t the column indices, row-start bits
// and first ordinal of its next tile are already in flight. Per tile the
// validation is an LDS read; only effective entries load their value and
// gather x, and the row of every start in the lane is fetched together with
// them (the ordinal map).
constexpr int kC5LdsThreads = 1024;
constexpr int kC5LdsWords = 32768;  // 128 KiB: n up to 2^20

template <int DT>
__global__ __launch_bounds__(kC5LdsThreads) void k_c5_spmspv_lds(
    int64_t ntiles, int32_t nnz, int32_t nwords, const int32_t* __restrict__ col,
    const typename SR<DT>::V* __restrict__ vals, const uint32_t* __restrict__ flags,
    const int32_t* __restrict__ tile_start, const int32_t* __restrict__ nz_rows,
    const typename SR<DT>::X* __restrict__ x, const uint32_t* __restrict__ bits, typename SR<DT>::Y* __restrict__ y,
    typename SR<DT>::Acc* __restrict__ lead, typename SR<DT>::Acc* __restrict__ trail) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    extern __shared__ __align__(16) uint32_t s_bits[];
    const int nvec = nwords >> 2;
    for (int w = threadIdx.x; w < nvec; w += kC5LdsThreads)
        reinterpret_cast<uint4*>(s_bits)[w] = reinterpret_cast<const uint4*>(bits)[w];
    for (int w = (nvec << 2) + (int)threadIdx.x; w < nwords; w += kC5LdsThreads) s_bits[w] = bits[w];
    __syncthreads();
    constexpr int kWaves = kC5LdsThreads / kWave;
    const int lane = lane_id();
    const int64_t stride = (int64_t)gridDim.x * kWaves;
    int64_t t = (int64_t)blockIdx.x * kWaves + threadIdx.x / kWave;  // uniform over the wave
    int cn[kC5Sigma];
    uint32_t fln = 0;
    int32_t tsn = 0;
    if (t < ntiles) {
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j) cn[j] = col[t * kC5Tile + j * kWave + lane];
        fln = flags[t * kWave + lane];
        tsn = tile_start[t];
    }
    for (; t < ntiles; t += stride) {
        int c[kC5Sigma];
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j) c[j] = cn[j];
        const uint32_t fl = fln;
        const int64_t base = t * kC5Tile;
        const int64_t first = base + (int64_t)lane * kC5Sigma;
        const int nfl = __popc(fl);
        const int ord0 = tsn + wave_incl_scan(nfl) - nfl;  // ordinal of the lane's first row start
        bool on[kC5Sigma];
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j)
            on[j] = first + j < nnz && ((s_bits[c[j] >> 5] >> (c[j] & 31)) & 1u);
        typename S::V a[kC5Sigma];
        typename S::X b[kC5Sigma];
        int32_t row[kC5Sigma];  // the row that starts at the lane's entry j
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j) a[j] = on[j] ? S::val(vals, base + j * kWave + lane) : (typename S::V)0;
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j) b[j] = on[j] ? S::xval(x, c[j]) : (typename S::X)0;
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j)
            row[j] = ((fl >> j) & 1u) ? nz_rows[ord0 + __popc(fl & ((1u << j) - 1u))] : 0;
        // the next tile's indices go out before this tile's sums wait
        const int64_t tn = t + stride;
        if (tn < ntiles) {
#pragma unroll
            for (int j = 0; j < kC5Sigma; ++j) cn[j] = col[tn * kC5Tile + j * kWave + lane];
            fln = flags[tn * kWave + lane];
            tsn = tile_start[tn];
        }
        Acc run = S::zero(), head = S::zero();
        bool seen = false;
        int32_t cur = 0;  // the row of the lane's latest start
#pragma unroll
        for (int j = 0; j < kC5Sigma; ++j) {
            if ((fl >> j) & 1u) {
                if (seen)
                    y[cur] = S::out(run);  // a row that starts and ends in this lane
                else
                    head = run;
                seen = true;
                cur = row[j];
                run = S::zero();
            }
            if (on[j]) run = S::fma(a[j], b[j], run);
        }
        if (!seen) head = run;
        Acc v = head;
        int f = seen ? 1 : 0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const Acc vo = shfl_down(v, d);
            const int fo = shfl_down(f, d);
            if (lane + d < kWave && !f) {
                v = S::add(v, vo);
                f = fo;
            }
        }
        const Acc vn = shfl_down(v, 1);
        const int fn = shfl_down(f, 1);
        if (seen) {
            const Acc tot = lane + 1 < kWave ? S::add(run, vn) : run;
            if (lane + 1 < kWave && fn)
                y[cur] = S::out(tot);
            else
                trail[t] = tot;  // the tile's last start: the row is still open
        }
        if (lane == 0) lead[t] = v;
    }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void k_c5_fixup(int64_t ntiles, const int32_t* __restrict__ tile_start,
                                                     const int32_t* __restrict__ nz_rows,
                                                     const typename SR<DT>::Acc* __restrict__ lead,
                                                     const typename SR<DT>::Acc* __restrict__ trail, int32_t nempty,
                                                     const int32_t* __restrict__ empty_rows,
                                                     typename SR<DT>::Y* __restrict__ y,
                                                     uint32_t* __restrict__ clear_bits, int32_t clear_words) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nempty; i += stride)
        y[empty_rows[i]] = S::out(S::zero());
    // the bitvector SpMSpV leaves the bitvector it read clean for the next call
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < clear_words; i += stride) clear_bits[i] = 0u;
    const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (t >= ntiles) return;
    const int32_t s1 = tile_start[t + 1];
    if (s1 == tile_start[t]) return;  // no row start here: this tile's sum is a lead
    const int lane = lane_id();
    Acc acc = trail[t];
    for (int64_t u0 = t + 1; u0 < ntiles; u0 += kWave) {
        const int64_t u = u0 + lane;
        const bool in = u < ntiles;
        const bool through = in && tile_start[u + 1] == tile_start[u];  // no start: the row runs on
        const uint64_t stop = __ballot(!through);
        const int last = stop ? __ffsll((unsigned long long)stop) - 1 : kWave - 1;
        Acc part = in && lane <= last ? lead[u] : S::zero();
        part = group_reduce<DT, kWave>(part);
        acc = S::add(acc, part);
        if (stop) break;
    }
    if (lane == 0) y[nz_rows[s1 - 1]] = S::out(acc);
}

// ------------------------------------------------------------------ host
void csr5_free(Csr5Mat* C) {
    void* ptrs[] = {C->col, C->vals, C->flags, C->tile_start, C->nz_rows, C->empty_rows, C->lead, C->trail};
    for (void* p : ptrs)
        if (p) hipFree(p);
    *C = Csr5Mat{};
}

int64_t csr5_cells(int32_t nnz) { return ceil_div((int64_t)nnz, kC5Tile) * kC5Tile; }

spx_status csr5_build(const spx_csr& A, const int32_t* rp, Csr5Mat* out, hipStream_t s) {
    Csr5Mat C;
    C.m = A.m;
    C.nnz = A.nnz;
    C.ntiles = ceil_div((int64_t)A.nnz, kC5Tile);
    C.cells = C.ntiles * kC5Tile;
    // row-start bits, tile ordinals and the row lists, from row_ptr
    std::vector<uint32_t> flags((size_t)C.ntiles * kWave, 0u);
    std::vector<int32_t> tile_start((size_t)C.ntiles + 1, 0);
    std::vector<int32_t> nz, empty;
    nz.reserve((size_t)A.m);
    for (int32_t r = 0; r < A.m; ++r) {
        if (rp[r + 1] > rp[r]) {
            const int64_t k = rp[r];
            const int64_t t = k / kC5Tile;
            const int w = (int)(k - t * kC5Tile);
            flags[(size_t)(t * kWave + w / kC5Sigma)] |= 1u << (w % kC5Sigma);
            nz.push_back(r);
        } else {
            empty.push_back(r);
        }
    }
    size_t q = 0;
    for (int64_t t = 0; t <= C.ntiles; ++t) {
        const int64_t pos = t * kC5Tile;
        while (q < nz.size() && rp[nz[q]] < pos) ++q;
        tile_start[(size_t)t] = (int32_t)q;
    }
    C.nonempty = (int32_t)nz.size();
    C.nempty = (int32_t)empty.size();
    const int vs = value_size(A.dtype);
    const size_t cells = (size_t)std::max<int64_t>(1, C.cells);
    const size_t tiles = (size_t)std::max<int64_t>(1, C.ntiles);
    auto alloc = [](void** p, size_t bytes) { return hipMalloc(p, std::max<size_t>(bytes, 4)) == hipSuccess; };
    if (!alloc((void**)&C.col, cells * 4) || (vs > 0 && !alloc(&C.vals, cells * vs)) ||
        !alloc((void**)&C.flags, tiles * kWave * 4) || !alloc((void**)&C.tile_start, (tiles + 1) * 4) ||
        !alloc((void**)&C.nz_rows, nz.size() * 4) || !alloc((void**)&C.empty_rows, empty.size() * 4) ||
        !alloc(&C.lead, tiles * 8) || !alloc(&C.trail, tiles * 8)) {
        csr5_free(&C);
        return fail(SPX_ERR_ALLOC, "CSR5 allocation failed");
    }
    bool ok = hipMemcpyAsync(C.flags, flags.data(), flags.size() * 4, hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(C.tile_start, tile_start.data(), tile_start.size() * 4, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              (nz.empty() ||
               hipMemcpyAsync(C.nz_rows, nz.data(), nz.size() * 4, hipMemcpyHostToDevice, s) == hipSuccess) &&
              (empty.empty() ||
               hipMemcpyAsync(C.empty_rows, empty.data(), empty.size() * 4, hipMemcpyHostToDevice, s) == hipSuccess);
    if (ok && C.cells > 0) {
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(C.cells, kBlock), 8192));
        k_c5_cols<<<grid, kBlock, 0, s>>>(C.cells, A.nnz, A.col_idx, C.col);
        ok = hipGetLastError() == hipSuccess;
    }
    // the host vectors must outlive the copies
    ok = ok && hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        csr5_free(&C);
        return fail(SPX_ERR_HIP, "CSR5 build");
    }
    *out = C;
    return csr5_refresh(*out, A, s);
}

spx_status csr5_refresh(const Csr5Mat& C, const spx_csr& A, hipStream_t s) {
    const int vs = value_size(A.dtype);
    if (vs == 0 || C.cells == 0) return SPX_OK;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(C.cells, kBlock), 8192));
    if (vs == 4)
        k_c5_vals<uint32_t><<<grid, kBlock, 0, s>>>(C.cells, A.nnz, (const uint32_t*)A.vals, (uint32_t*)C.vals);
    else
        k_c5_vals<uint64_t><<<grid, kBlock, 0, s>>>(C.cells, A.nnz, (const uint64_t*)A.vals, (uint64_t*)C.vals);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

template <int DT>
static spx_status csr5_spmv_t(const Csr5Mat& C, const void* x, void* y, hipStream_t s) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    auto* yv = (typename S::Y*)y;
    if (C.ntiles > 0) {
        const unsigned grid = (unsigned)ceil_div(C.ntiles, kWavesPerBlock);
        k_c5_spmv<DT><<<grid, kBlock, 0, s>>>(C.ntiles, C.nnz, C.col, (const typename S::V*)C.vals, C.flags,
                                              C.tile_start, C.nz_rows, (const typename S::X*)x, yv, (Acc*)C.lead,
                                              (Acc*)C.trail);
        SPX_HIP(hipGetLastError());
    }
    const int64_t blocks = std::max<int64_t>(
        {(int64_t)1, ceil_div(C.ntiles, kWavesPerBlock), std::min<int64_t>(ceil_div(C.nempty, kBlock), 4096)});
    k_c5_fixup<DT><<<(unsigned)blocks, kBlock, 0, s>>>(C.ntiles, C.tile_start, C.nz_rows, (const Acc*)C.lead,
                                                       (const Acc*)C.trail, C.nempty, C.empty_rows, yv, nullptr, 0);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

bool csr5_lds_fits(int32_t n) { return n >= 0 && (int64_t)(n + 31) / 32 <= kC5LdsWords; }

template <int DT>
static spx_status csr5_spmspv_t(const Csr5Mat& C, int32_t n, const void* x, uint32_t* bits, void* y,
                                hipStream_t s) {
    using S = SR<DT>;
    using Acc = typename S::Acc;
    auto* yv = (typename S::Y*)y;
    const int32_t nwords = (n + 31) / 32;
    if (C.ntiles > 0) {
        static int cus = 0;
        if (!cus) {
            int dev = 0;
            SPX_HIP(hipGetDevice(&dev));
            SPX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            cus = std::max(cus, 1);
        }
        const size_t lds = (size_t)std::max(nwords, 4) * 4;
        SPX_HIP(hipFuncSetAttribute((const void*)k_c5_spmspv_lds<DT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
        const unsigned grid = (unsigned)std::min<int64_t>(cus, ceil_div(C.ntiles, kC5LdsThreads / kWave));
        k_c5_spmspv_lds<DT><<<grid, kC5LdsThreads, lds, s>>>(C.ntiles, C.nnz, nwords, C.col,
                                                             (const typename S::V*)C.vals, C.flags, C.tile_start,
                                                             C.nz_rows, (const typename S::X*)x, bits, yv,
                                                             (Acc*)C.lead, (Acc*)C.trail);
        SPX_HIP(hipGetLastError());
    }
    const int64_t blocks = std::max<int64_t>({(int64_t)1, ceil_div(C.ntiles, kWavesPerBlock),
                                              std::min<int64_t>(ceil_div(C.nempty, kBlock), 4096),
                                              std::min<int64_t>(ceil_div(nwords, kBlock), 4096)});
    k_c5_fixup<DT><<<(unsigned)blocks, kBlock, 0, s>>>(C.ntiles, C.tile_start, C.nz_rows, (const Acc*)C.lead,
                                                       (const Acc*)C.trail, C.nempty, C.empty_rows, yv, bits, nwords);
    SPX_HIP(hipGetLastError());
    return SPX_OK;
}

spx_status csr5_spmspv(const Csr5Mat& C, int dtype, int32_t n, const void* x, uint32_t* bits, void* y,
                       hipStream_t s) {
    if (C.m == 0) return SPX_OK;
    if (!csr5_lds_fits(n)) return fail(SPX_ERR_UNSUPPORTED, "CSR5 SpMSpV: n above 2^20");
    if (((uintptr_t)bits & 15) != 0) return fail(SPX_ERR_ARG, "CSR5 SpMSpV: bitvector not 16-byte aligned");
    switch (dtype) {
        case SPX_F32: return csr5_spmspv_t<SPX_F32>(C, n, x, bits, y, s);
        case SPX_F64: return csr5_spmspv_t<SPX_F64>(C, n, x, bits, y, s);
        case SPX_I32: return csr5_spmspv_t<SPX_I32>(C, n, x, bits, y, s);
        case SPX_BOOL: return csr5_spmspv_t<SPX_BOOL>(C, n, x, bits, y, s);
        case SPX_F32_MINPLUS: return csr5_spmspv_t<SPX_F32_MINPLUS>(C, n, x, bits, y, s);
    }
    return fail(SPX_ERR_DTYPE, "CSR5 SpMSpV: unknown dtype");
}

spx_status csr5_spmv(const Csr5Mat& C, int dtype, const void* x, void* y, hipStream_t s) {
    if (C.m == 0) return SPX_OK;
    switch (dtype) {
        case SPX_F32: return csr5_spmv_t<SPX_F32>(C, x, y, s);
        case SPX_F64: return csr5_spmv_t<SPX_F64>(C, x, y, s);
        case SPX_I32: return csr5_spmv_t<SPX_I32>(C, x, y, s);
        case SPX_BOOL: return csr5_spmv_t<SPX_BOOL>(C, x, y, s);
        case SPX_F32_MINPLUS: return csr5_spmv_t<SPX_F32_MINPLUS>(C, x, y, s);
    }
    return fail(SPX_ERR_DTYPE, "CSR5: unknown dtype");
}

}  // namespace spx
