// HIP kernels for gfx950 (MI355X): block permute/fuse/split, the grouped
// sector GEMM on MFMA (FP32 and BF16 with FP32 accumulation), and the SU(2)
// recoupling of reduced blocks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "kernels.hpp"

namespace sym {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// element conversion
// ---------------------------------------------------------------------------

// FP32 -> BF16, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<uint16_t>((u >> 16) | 0x0040u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

template <typename Ti, typename To>
struct Conv;
template <>
struct Conv<float, float> {
    __device__ static float f(float x) { return x; }
};
template <>
struct Conv<float, uint16_t> {
    __device__ static uint16_t f(float x) { return f32_to_bf16(x); }
};
template <>
struct Conv<uint16_t, uint16_t> {
    __device__ static uint16_t f(uint16_t x) { return x; }
};
template <>
struct Conv<uint16_t, float> {
    __device__ static float f(uint16_t x) { return bf16_to_f32(x); }
};

// sign change of a converted element (exact: flips the sign bit)
__device__ __forceinline__ float flip(float x, int neg) { return neg ? -x : x; }
__device__ __forceinline__ uint16_t flip(uint16_t x, int neg) {
    return static_cast<uint16_t>(x ^ (neg ? 0x8000u : 0u));
}

// floor(n / d) for 0 <= n < 2^31 from the divisor's multiplier and shift
__device__ __forceinline__ int div_by(int n, uint32_t mag, int shf) {
    return static_cast<int>((static_cast<uint64_t>(static_cast<uint32_t>(n)) * mag) >> (31 + shf));
}

// ---------------------------------------------------------------------------
// K2/K3: block permute (fuse, split, reorder).  Each workgroup walks its own
// range of tasks; a task is a slice of one block copy.  Threads run along the
// destination's innermost dimension, so stores are coalesced; loads are
// coalesced whenever the copy keeps the source's innermost dimension.
// ---------------------------------------------------------------------------
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_permute(const CopyOp* __restrict__ ops, const CopyTask* __restrict__ tasks,
                                                 const int32_t* __restrict__ wg_begin, PtrTable bufs) {
    const int w = blockIdx.x;
    const int t_lo = wg_begin[w], t_hi = wg_begin[w + 1];
    for (int ti = t_lo; ti < t_hi; ++ti) {
        const CopyTask t = tasks[ti];
        const CopyOp& op = ops[t.op];
        const Ti* __restrict__ src = static_cast<const Ti*>(bufs.p[op.src_buf]) + op.src_off;
        To* __restrict__ dst = static_cast<To*>(const_cast<void*>(bufs.p[op.dst_buf])) + op.dst_off;
        const int nd = op.ndim;
        const int inner = op.size[kMaxCopyDims - 1];
        const int64_t s_in = op.sstride[kMaxCopyDims - 1], d_in = op.dstride[kMaxCopyDims - 1];
        const int end = t.start + t.count;
        // U independent elements per thread per pass (16 bytes of 2-byte
        // elements): all loads are in flight before the first store waits
        constexpr int U = sizeof(Ti) == 2 ? 8 : 4;
        for (int base = t.start; base < end; base += 256 * U) {
            Ti v[U];
            int64_t dofs[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = base + static_cast<int>(threadIdx.x) + u * 256;
                ok[u] = e < end;
                const int ee = ok[u] ? e : t.start;
                int rem = div_by(ee, op.mag[kMaxCopyDims - 1], op.shf[kMaxCopyDims - 1]);
                const int i0 = ee - rem * inner;
                int64_t so = i0 * s_in, dof = i0 * d_in;
                for (int d = kMaxCopyDims - 2; d >= kMaxCopyDims - nd; --d) {
                    const int q = div_by(rem, op.mag[d], op.shf[d]);
                    const int i = rem - q * op.size[d];
                    rem = q;
                    so += i * op.sstride[d];
                    dof += i * op.dstride[d];
                }
                dofs[u] = dof;
                v[u] = src[so];
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) dst[dofs[u]] = flip(Conv<Ti, To>::f(v[u]), op.neg);
        }
    }
}

// Row copy: the task's source elements form one contiguous run.  They are
// staged through LDS with 16-byte loads from 16-byte aligned addresses (a
// range-checked buffer resource ends at the source buffer, so the loads past
// the run's last element read zeros instead of memory beyond it), then every
// destination row is written in 16-byte aligned chunks gathered from LDS;
// the partial chunks at either end of a row take element stores.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

template <typename To>
struct Pack;
template <>
struct Pack<float> {
    static constexpr int V = 4;
    __device__ static u32x4_t f(const float (&v)[4]) {
        return u32x4_t{__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]), __float_as_uint(v[3])};
    }
};
template <>
struct Pack<uint16_t> {
    static constexpr int V = 8;
    __device__ static u32x4_t f(const uint16_t (&v)[8]) {
        u32x4_t r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = static_cast<uint32_t>(v[2 * i]) | (static_cast<uint32_t>(v[2 * i + 1]) << 16);
        return r;
    }
};

// threads of a row-copy workgroup: on the batched BF16 fuse (32 members,
// A side plus B side) 512 measured 1 % faster than 256; staging 16384
// instead of 8192 source elements per task gained another 0.5 % but doubles
// the FP32 stage, 4096 lost 0.6 %
constexpr int kCrThreads = 512;
template <typename Ti, typename To>
__global__ __launch_bounds__(kCrThreads) void k_copy_rows(const CopyOp* __restrict__ ops, const RowTask* __restrict__ tasks,
                                                   int n_tasks, PtrTable bufs) {
    constexpr int VI = 16 / sizeof(Ti);
    constexpr int VO = Pack<To>::V;
    constexpr int I = kMaxCopyDims - 1;
    __shared__ __attribute__((aligned(16))) Ti stage[kRowStage + 2 * VI];
    for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
        const RowTask t = tasks[ti];
        const CopyOp& op = ops[t.op];
        const Ti* __restrict__ src = static_cast<const Ti*>(bufs.p[op.src_buf]);
        To* __restrict__ dst = static_cast<To*>(const_cast<void*>(bufs.p[op.dst_buf]));
        const int L = op.size[I];
        const int64_t ldd = op.ndim > 1 ? op.dstride[I - 1] : 0;
        const int64_t s0 = op.src_off + static_cast<int64_t>(t.row0) * L + t.col0;
        const int n = t.nrows == 1 ? t.ncols : t.nrows * L;
        // stage source elements [a0, s0 + n) at LDS index (element - a0)
        const bool vec_src = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
        const int64_t a0 = vec_src ? (s0 & ~static_cast<int64_t>(VI - 1)) : s0;
        if (vec_src) {
            const int span = static_cast<int>(s0 + n - a0);
            const int64_t avail = op.src_len - a0;
            const int lim = static_cast<int>(avail < span + VI ? avail : span + VI);
            // the range check works on whole 4-byte words: a 2-byte element
            // sharing its word with the end of the buffer is loaded below
            const int full = static_cast<int>(lim * sizeof(Ti)) & ~3;
            const __amdgpu_buffer_rsrc_t r =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<Ti*>(src + a0), static_cast<short>(0), full, 0x00020000);
            const int nvec = (span + VI - 1) / VI;
            const int e_full = full / static_cast<int>(sizeof(Ti));
            for (int v = threadIdx.x; v < nvec; v += kCrThreads) {
                reinterpret_cast<u32x4_t*>(stage)[v] =
                    __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(r, v * 16, 0, 0));
                for (int e = v * VI > e_full ? v * VI : e_full; e < (v + 1) * VI && e < lim; ++e)
                    stage[e] = src[a0 + e];
            }
        } else {
            for (int e = threadIdx.x; e < n; e += kCrThreads) stage[e] = src[s0 + e];
        }
        __syncthreads();
        const int off = static_cast<int>(s0 - a0);
        const int cols = t.ncols;
        const int maxch = (cols + 2 * VO - 2) / VO;
        const int items = t.nrows * maxch;
        const bool vec_dst = (reinterpret_cast<uintptr_t>(dst) & 15) == 0;
        const float inv = 1.f / static_cast<float>(maxch);
        for (int it = threadIdx.x; it < items; it += kCrThreads) {
            int q = static_cast<int>(static_cast<float>(it) * inv);
            int j = it - q * maxch;
            if (j < 0) {
                --q;
                j += maxch;
            } else if (j >= maxch) {
                ++q;
                j -= maxch;
            }
            const int64_t d0 = op.dst_off + static_cast<int64_t>(t.row0 + q) * ldd + t.col0;
            const int delta = vec_dst ? static_cast<int>(d0 & (VO - 1)) : 0;
            const int c_lo = j * VO - delta;
            const Ti* row = stage + off + q * L;
            if (vec_dst && c_lo >= 0 && c_lo + VO <= cols) {
                To v[VO];
#pragma unroll
                for (int u = 0; u < VO; ++u) v[u] = flip(Conv<Ti, To>::f(row[c_lo + u]), op.neg);
                *reinterpret_cast<u32x4_t*>(dst + d0 + c_lo) = Pack<To>::f(v);
            } else {
#pragma unroll
                for (int u = 0; u < VO; ++u) {
                    const int c = c_lo + u;
                    if (c >= 0 && c < cols) dst[d0 + c] = flip(Conv<Ti, To>::f(row[c]), op.neg);
                }
            }
        }
        __syncthreads();   // the stage is free for the next task
    }
}

hipError_t launch_copy_rows(int src_dtype, int dst_dtype, const CopyOp* ops, const RowTask* tasks, int32_t n_tasks,
                            int32_t n_wg, const PtrTable& bufs, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    if (n_wg <= 0) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(n_wg)), block(kCrThreads);
    if (src_dtype == 0 && dst_dtype == 0)
        hipLaunchKernelGGL((k_copy_rows<float, float>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    else if (src_dtype == 0 && dst_dtype == 1)
        hipLaunchKernelGGL((k_copy_rows<float, uint16_t>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    else if (src_dtype == 1 && dst_dtype == 1)
        hipLaunchKernelGGL((k_copy_rows<uint16_t, uint16_t>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    else
        hipLaunchKernelGGL((k_copy_rows<uint16_t, float>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    return hipGetLastError();
}

// Transposing block copy: the source is contiguous along dim tj, the
// destination along the innermost dim.  A 64 x 64 tile is read with lanes
// running along the source's contiguous dim, staged in LDS (row pitch 65 keeps
// the transposed reads free of bank conflicts) and written with lanes running
// along the destination's contiguous dim, so both sides stay coalesced.
template <typename Ti, typename To>
__device__ __forceinline__ void tile_copy(const CopyOp* __restrict__ ops, const TileTask t, const PtrTable& bufs,
                                          Ti (&tile)[kTile][kTile + 1]) {
    const CopyOp& op = ops[t.op];
    const Ti* __restrict__ src = static_cast<const Ti*>(bufs.p[op.src_buf]) + op.src_off;
    To* __restrict__ dst = static_cast<To*>(const_cast<void*>(bufs.p[op.dst_buf])) + op.dst_off;
    constexpr int I = kMaxCopyDims - 1;
    const int J = op.tj;
    int64_t so = 0, dof = 0;
    int rem = t.outer;
    for (int d = kMaxCopyDims - 2; d >= kMaxCopyDims - op.ndim; --d) {
        if (d == J) continue;
        const int q = div_by(rem, op.mag[d], op.shf[d]);
        const int i = rem - q * op.size[d];
        rem = q;
        so += i * op.sstride[d];
        dof += i * op.dstride[d];
    }
    const int nI = op.size[I], nJ = op.size[J];
    const int64_t sI = op.sstride[I], dI = op.dstride[I], sJ = op.sstride[J], dJ = op.dstride[J];
    const int i0 = t.it * kTile, j0 = t.jt * kTile;
    const int lo = threadIdx.x & 63, hi = threadIdx.x >> 6;
#pragma unroll 4
    for (int r = 0; r < kTile / 4; ++r) {
        const int i = i0 + hi + 4 * r, j = j0 + lo;
        if (i < nI && j < nJ) tile[i - i0][j - j0] = src[so + i * sI + j * sJ];
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kTile / 4; ++r) {
        const int j = j0 + hi + 4 * r, i = i0 + lo;
        if (i < nI && j < nJ) dst[dof + i * dI + j * dJ] = flip(Conv<Ti, To>::f(tile[i - i0][j - j0]), op.neg);
    }
}

// Vectorized transposing copy for tiles whose destination rows are
// contiguous (unit stride along the destination's inner dim).  A tile is
// TI (destination-contiguous dim) x kTile (source-contiguous dim); TI is
// long so that a tile writes long destination row segments and few partial
// cache lines.  Each source row of the tile is staged with 16-byte loads
// from its aligned-down start; row r sits at LDS column rot(r) + off[r],
// where the rotation rot(r) = VI ((r / 8) mod 8) puts rows 8 apart on
// different banks.  All of a thread's source loads are issued before its
// first LDS write.  Destination rows are written in 16-byte aligned chunks,
// eight lanes per row on eight consecutive chunks (128 contiguous bytes),
// each chunk gathered down an LDS column; element stores only at the ends.
// The source is read through one range-checked buffer resource per tile
// that ends at the source buffer.
template <typename Ti>
struct TransposeShape {
    static constexpr int VI = 16 / sizeof(Ti);
    static constexpr int VC = vtile_cols(sizeof(Ti));       // tile columns (source-contiguous)
    static constexpr int NV = (VC + 2 * VI - 2) / VI;       // vectors that cover one source row segment
    static constexpr int RW = VC + 2 * VI + 7 * VI;          // staged row width incl. rotation room
    static constexpr int TI = vtile_rows(sizeof(Ti));
    static constexpr size_t lds_bytes = static_cast<size_t>(TI) * RW * sizeof(Ti) + TI * sizeof(int);
};

// threads of a transposing workgroup: the LDS tile (70 KB for BF16) allows
// two workgroups per CU, so more threads per workgroup are more loads in
// flight per CU; on the batched BF16 fuse 512 measured 2 % faster than 256
// (both with the next tile's loads issued before the current tile is
// written out, itself 2 % faster than without), 1024 0.5 % slower than 512
constexpr int kTvThreads = 512;
template <typename Ti, typename To, bool MERGED>
__global__ __launch_bounds__(kTvThreads) void k_transpose_vec(const CopyOp* __restrict__ ops,
                                                       const TileTask* __restrict__ tasks, int n_tasks,
                                                       PtrTable bufs) {
    using Sh = TransposeShape<Ti>;
    constexpr int VI = Sh::VI, NV = Sh::NV, RW = Sh::RW, TI = Sh::TI, VC = Sh::VC;
    constexpr int VO = Pack<To>::V;
    constexpr int NC = (TI + 2 * VO - 2) / VO;      // chunks that cover one destination row segment
    constexpr int NH = (NC + 7) / 8;                // groups of eight chunks
    constexpr int NLD = (TI * NV + kTvThreads - 1) / kTvThreads;   // source vectors per thread
    constexpr int NW = kTvThreads / 64;                             // waves
    constexpr int I = kMaxCopyDims - 1;
    static_assert((RW * sizeof(Ti)) % 16 == 0, "LDS rows must stay 16-byte aligned");
    extern __shared__ u32x4_t lds_raw[];
    Ti* tile = reinterpret_cast<Ti*>(lds_raw);
    int* row_off = reinterpret_cast<int*>(tile + TI * RW);
    auto rot = [](int r) { return VI * ((r >> 3) & 7); };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // everything one tile's staging and write phase need
    struct Tile {
        const CopyOp* op;
        const Ti* src;
        To* dst;
        int64_t so, dof, base;
        int i0, j0, ni, nj, lim, e_full, nIlo, nJlo;
        int64_t sI, sIhi, dJ, dJhi;
        __amdgpu_buffer_rsrc_t rs;
    };
    auto setup = [&](int ti, Tile& c) {
        const TileTask t = tasks[ti];
        const CopyOp& op = ops[t.op];
        c.op = &op;
        c.src = static_cast<const Ti*>(bufs.p[op.src_buf]);
        c.dst = static_cast<To*>(const_cast<void*>(bufs.p[op.dst_buf]));
        const int J = op.tj;
        c.so = op.src_off;
        c.dof = op.dst_off;
        int rem = t.outer;
        for (int d = kMaxCopyDims - 2; d >= kMaxCopyDims - op.ndim; --d) {
            if (d == J || (MERGED && (d == op.ihi || d == op.jhi))) continue;
            const int q = div_by(rem, op.mag[d], op.shf[d]);
            const int i = rem - q * op.size[d];
            rem = q;
            c.so += i * op.sstride[d];
            c.dof += i * op.dstride[d];
        }
        // tile rows i (destination-contiguous, index i_lo + size[I] i_hi)
        // and columns j (source-contiguous, j_lo + size[J] j_hi)
        // (MERGED: ops with ihi or jhi set; the launch of the others never
        // divides)
        c.nIlo = op.size[I];
        c.nJlo = op.size[J];
        const int nI = MERGED && op.ihi >= 0 ? c.nIlo * op.size[op.ihi] : c.nIlo;
        const int nJ = MERGED && op.jhi >= 0 ? c.nJlo * op.size[op.jhi] : c.nJlo;
        c.sI = op.sstride[I];
        c.sIhi = MERGED && op.ihi >= 0 ? op.sstride[op.ihi] : 0;
        c.dJ = op.dstride[J];
        c.dJhi = MERGED && op.jhi >= 0 ? op.dstride[op.jhi] : 0;
        c.i0 = t.it * TI;
        c.j0 = t.jt * VC;
        c.ni = min(TI, nI - c.i0);
        c.nj = min(VC, nJ - c.j0);
        // row r of the tile: source elements [so + src_row(i0 + r) + j0, + nj);
        // the lowest row start is that of the first row, or of i_lo = 0 in
        // the tile's first i_hi when the tile wraps past the end of i_lo
        const int h0 = MERGED ? div_by(c.i0, op.mag[I], op.shf[I]) : 0;
        const int64_t first =
            (c.i0 - h0 * c.nIlo + c.ni > c.nIlo ? int64_t{0} : (c.i0 - h0 * c.nIlo) * c.sI) + h0 * c.sIhi;
        c.base = (c.so + first + c.j0) & ~static_cast<int64_t>(VI - 1);
        const int64_t avail = op.src_len - c.base;
        const int64_t cap = (int64_t{1} << 30) / static_cast<int64_t>(sizeof(Ti));
        c.lim = static_cast<int>(avail < cap ? avail : cap);
        const int full = static_cast<int>(c.lim * sizeof(Ti)) & ~3;
        c.e_full = full / static_cast<int>(sizeof(Ti));
        c.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<Ti*>(c.src + c.base), static_cast<short>(0), full,
                                                 0x00020000);
    };
    auto src_row = [&](const Tile& c, int i) -> int64_t {   // source offset of row i
        if constexpr (!MERGED) return i * c.sI;
        const int h = div_by(i, c.op->mag[I], c.op->shf[I]);
        return (i - h * c.nIlo) * c.sI + h * c.sIhi;
    };
    auto dst_row = [&](const Tile& c, int j) -> int64_t {   // destination offset of column j
        if constexpr (!MERGED) return j * c.dJ;
        const int h = div_by(j, c.op->mag[c.op->tj], c.op->shf[c.op->tj]);
        return (j - h * c.nJlo) * c.dJ + h * c.dJhi;
    };
    // item it = (row r, vector v)
    auto item = [&](const Tile& c, int it, int& r, int& v, int& off, int& e0) {
        r = it / NV;
        v = it - r * NV;
        if (it >= TI * NV || r >= c.ni) return false;
        const int64_t start = c.so + src_row(c, c.i0 + r) + c.j0;
        const int64_t a = start & ~static_cast<int64_t>(VI - 1);
        off = static_cast<int>(start - a);
        e0 = static_cast<int>(a - c.base) + v * VI;   // element index from the resource base
        return true;
    };
    u32x4_t ld[NLD];
    auto issue = [&](const Tile& c) {
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            int r, v, off, e0;
            ld[u] = u32x4_t{0u, 0u, 0u, 0u};
            if (item(c, static_cast<int>(threadIdx.x) + kTvThreads * u, r, v, off, e0) && v * VI < off + c.nj)
                ld[u] = __builtin_bit_cast(u32x4_t, __builtin_amdgcn_raw_buffer_load_b128(
                                                        c.rs, e0 * static_cast<int>(sizeof(Ti)), 0, 0));
        }
    };
    auto stage = [&](const Tile& c) {
#pragma unroll
        for (int u = 0; u < NLD; ++u) {
            int r, v, off, e0;
            if (!item(c, static_cast<int>(threadIdx.x) + kTvThreads * u, r, v, off, e0)) continue;
            if (v == 0) row_off[r] = rot(r) + off;
            if (v * VI >= off + c.nj) continue;
            Ti* row = tile + r * RW + rot(r);
            reinterpret_cast<u32x4_t*>(row)[v] = ld[u];
            for (int e = e0 > c.e_full ? e0 : c.e_full; e < e0 + VI && e < c.lim; ++e)
                row[v * VI + (e - e0)] = c.src[c.base + e];
        }
    };
    auto emit = [&](const Tile& c) {
        const bool vec_dst = (reinterpret_cast<uintptr_t>(c.dst) & 15) == 0;
        const int neg = c.op->neg;
        // wave item (g, h): lane (jj, cc) writes chunk 8 h + cc of destination row j0 + 8 g + jj
        for (int wi = wave; wi < (VC / 8) * NH; wi += NW) {
            const int g = wi / NH, h = wi - g * NH;
            const int j = 8 * g + (lane >> 3), cc = 8 * h + (lane & 7);
            if (j >= c.nj || cc >= NC) continue;
            const int64_t d0 = c.dof + dst_row(c, c.j0 + j) + c.i0;
            const int delta = vec_dst ? static_cast<int>(d0 & (VO - 1)) : 0;
            const int c_lo = cc * VO - delta;
            if (c_lo >= c.ni || c_lo + VO <= 0) continue;
            if (vec_dst && c_lo >= 0 && c_lo + VO <= c.ni) {
                To v[VO];
#pragma unroll
                for (int u = 0; u < VO; ++u)
                    v[u] = flip(Conv<Ti, To>::f(tile[(c_lo + u) * RW + row_off[c_lo + u] + j]), neg);
                *reinterpret_cast<u32x4_t*>(c.dst + d0 + c_lo) = Pack<To>::f(v);
            } else {
#pragma unroll
                for (int u = 0; u < VO; ++u) {
                    const int r = c_lo + u;
                    if (r >= 0 && r < c.ni) c.dst[d0 + r] = flip(Conv<Ti, To>::f(tile[r * RW + row_off[r] + j]), neg);
                }
            }
        }
    };

    // software pipeline: the next tile's source loads are in flight while
    // this tile is written out
    int ti = blockIdx.x;
    if (ti >= n_tasks) return;
    Tile cur;
    setup(ti, cur);
    issue(cur);
    for (; ti < n_tasks; ti += gridDim.x) {
        stage(cur);
        __syncthreads();
        const int tn = ti + static_cast<int>(gridDim.x);
        Tile nxt = cur;
        if (tn < n_tasks) {
            setup(tn, nxt);
            issue(nxt);
        }
        emit(cur);
        __syncthreads();   // the tile is free for the next task
        cur = nxt;
    }
}

template <typename Ti, typename To, bool MERGED>
hipError_t launch_tv(const CopyOp* ops, const TileTask* tasks, int32_t n_tasks, int32_t n_wg, const PtrTable& bufs,
                     hipStream_t s) {
    constexpr size_t lds = TransposeShape<Ti>::lds_bytes;
    // once per process (a thread-safe static initialisation)
    static const hipError_t configured =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_transpose_vec<Ti, To, MERGED>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (configured != hipSuccess) return configured;
    hipLaunchKernelGGL((k_transpose_vec<Ti, To, MERGED>), dim3(static_cast<unsigned>(n_wg)), dim3(kTvThreads), lds, s, ops,
                       tasks, n_tasks, bufs);
    return hipGetLastError();
}

// Each workgroup walks tiles blockIdx.x, blockIdx.x + gridDim.x, ...
template <typename Ti, typename To>
__global__ __launch_bounds__(256) void k_permute_tiled(const CopyOp* __restrict__ ops, const TileTask* __restrict__ tasks,
                                                       int n_tasks, PtrTable bufs) {
    __shared__ Ti tile[kTile][kTile + 1];
    for (int ti = blockIdx.x; ti < n_tasks; ti += gridDim.x) {
        tile_copy<Ti, To>(ops, tasks[ti], bufs, tile);
        __syncthreads();   // every read of the tile is done before the next task writes it
    }
}

template <bool MERGED>
hipError_t launch_tv_types(int src_dtype, int dst_dtype, const CopyOp* ops, const TileTask* tasks, int32_t n_tasks,
                           int32_t n_wg, const PtrTable& bufs, hipStream_t s) {
    if (src_dtype == 0 && dst_dtype == 0) return launch_tv<float, float, MERGED>(ops, tasks, n_tasks, n_wg, bufs, s);
    if (src_dtype == 0 && dst_dtype == 1) return launch_tv<float, uint16_t, MERGED>(ops, tasks, n_tasks, n_wg, bufs, s);
    if (src_dtype == 1 && dst_dtype == 1)
        return launch_tv<uint16_t, uint16_t, MERGED>(ops, tasks, n_tasks, n_wg, bufs, s);
    return launch_tv<uint16_t, float, MERGED>(ops, tasks, n_tasks, n_wg, bufs, s);
}

hipError_t launch_transpose_vec(int src_dtype, int dst_dtype, bool merged, const CopyOp* ops, const TileTask* tasks,
                                int32_t n_tasks, int32_t n_wg, const PtrTable& bufs, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    if (n_wg <= 0) return hipErrorInvalidValue;
    return merged ? launch_tv_types<true>(src_dtype, dst_dtype, ops, tasks, n_tasks, n_wg, bufs, s)
                  : launch_tv_types<false>(src_dtype, dst_dtype, ops, tasks, n_tasks, n_wg, bufs, s);
}

hipError_t launch_permute_tiled(int src_dtype, int dst_dtype, const CopyOp* ops, const TileTask* tasks, int32_t n_tasks,
                                int32_t n_wg, const PtrTable& bufs, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    if (n_wg <= 0) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(n_wg)), block(256);
    if (src_dtype == 0 && dst_dtype == 0)
        hipLaunchKernelGGL((k_permute_tiled<float, float>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    else if (src_dtype == 0 && dst_dtype == 1)
        hipLaunchKernelGGL((k_permute_tiled<float, uint16_t>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    else if (src_dtype == 1 && dst_dtype == 1)
        hipLaunchKernelGGL((k_permute_tiled<uint16_t, uint16_t>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    else
        hipLaunchKernelGGL((k_permute_tiled<uint16_t, float>), grid, block, 0, s, ops, tasks, n_tasks, bufs);
    return hipGetLastError();
}

hipError_t launch_permute(int src_dtype, int dst_dtype, const CopyOp* ops, const CopyTask* tasks,
                          const int32_t* wg_begin, int32_t n_wg, const PtrTable& bufs, hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    dim3 grid(static_cast<unsigned>(n_wg)), block(256);
    if (src_dtype == 0 && dst_dtype == 0)
        hipLaunchKernelGGL((k_permute<float, float>), grid, block, 0, s, ops, tasks, wg_begin, bufs);
    else if (src_dtype == 0 && dst_dtype == 1)
        hipLaunchKernelGGL((k_permute<float, uint16_t>), grid, block, 0, s, ops, tasks, wg_begin, bufs);
    else if (src_dtype == 1 && dst_dtype == 1)
        hipLaunchKernelGGL((k_permute<uint16_t, uint16_t>), grid, block, 0, s, ops, tasks, wg_begin, bufs);
    else
        hipLaunchKernelGGL((k_permute<uint16_t, float>), grid, block, 0, s, ops, tasks, wg_begin, bufs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K4/K5/K6: persistent grouped GEMM over sector tiles.
//
// C[m][n] = sum_k A[m][k] B[n][k]; A rows and B rows are K-contiguous.  A
// workgroup of 4 waves owns an MT x NT tile of C; wave (wm, wn) owns an
// (MT/2) x (NT/2) sub-tile built from 32x32 MFMA blocks.  Operand tiles are
// staged through LDS in two buffers: the next K slice is fetched into
// registers while the current one feeds the MFMAs.
//
// Inside one MFMA the K index is a free relabelling as long as A and B agree:
// lanes 0-31 feed the first half of an LDS row slice and lanes 32-63 the
// second half, so every lane reads 16-byte vectors from LDS.
// ---------------------------------------------------------------------------

// Epilogue of a wave's (32 FM) x (32 FN) sub-tile starting at (mb, nb).  A
// 32x32 MFMA result leaves lane l with column (l & 31) and, in register
// 4*i+j, row 8*i + 4*(l >> 5) + j.  Plain outputs are row-major with ldc;
// indirect outputs go straight to their canonical block (see GemmProb).
template <int FM, int FN>
__device__ __forceinline__ void store_tile(const v16f (&acc)[FM][FN], const GemmProb& p, float* C,
                                           const EpiRow* __restrict__ rows, const EpiCol* __restrict__ cols, int mb,
                                           int nb, int h, int r32) {
    if (!p.indirect) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int col = nb + j * 32 + r32;
                if (col >= p.N) continue;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int row = mb + i * 32 + (q >> 2) * 8 + h * 4 + (q & 3);
                    if (row < p.M) C[static_cast<int64_t>(row) * p.ldc + col] = acc[i][j][q];
                }
            }
        return;
    }
    // canonical-block output: 32-bit offsets from the buffer base (the host
    // checks the bounds that make this exact) and range-checked buffer stores
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(C, static_cast<short>(0), 0x7fffffff, 0x00020000);
    EpiCol cj[FN];
    bool cok[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = nb + j * 32 + r32;
        cok[j] = col < p.N;
        cj[j] = cols[p.ci_off + (cok[j] ? col : 0)];
    }
    // branch-free (see store_tile_tab): elements outside the matrix get the
    // out-of-range offset 0x80000000 and the buffer store drops them
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int row = mb + i * 32 + (q >> 2) * 8 + h * 4 + (q & 3);
            const bool rok = row < p.M;
            const EpiRow ri = rows[p.ri_off + (rok ? row : p.M - 1)];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const uint32_t e = static_cast<uint32_t>(ri.r0 + cj[j].c0) +
                                   __umul24(static_cast<uint32_t>(ri.r1), static_cast<uint32_t>(cj[j].c1)) +
                                   __umul24(static_cast<uint32_t>(ri.r2), static_cast<uint32_t>(cj[j].c2));
                const uint32_t vo = (rok && cok[j]) ? e * 4u : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[i][j][q]), rc, vo, 0, 0);
            }
        }
}

// Canonical-block epilogue with the tile's row terms staged in LDS: tab[r]
// holds the EpiRow of tile row r (rows past M repeat the last row's terms),
// so no store waits on a memory load.  The code is branch-free: an element
// outside the matrix gets the out-of-range offset 0x80000000, which the
// buffer store drops; branches around each store would make the compiler
// wait for every store before the next (vector memory operations complete
// in order and its wait analysis is conservative across branches).  mt0: the
// tile's first row; ml: this wave's first row inside the tile.
template <int FM, int FN>
__device__ __forceinline__ void store_tile_tab(const v16f (&acc)[FM][FN], const GemmProb& p, float* C,
                                               const EpiRow* tab, const EpiCol* __restrict__ cols, int mt0, int ml,
                                               int nb, int h, int r32) {
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(C, static_cast<short>(0), 0x7fffffff, 0x00020000);
    EpiCol cj[FN];
    bool cok[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int col = nb + j * 32 + r32;
        cok[j] = col < p.N;
        cj[j] = cols[p.ci_off + (cok[j] ? col : 0)];
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int rl = ml + i * 32 + (q >> 2) * 8 + h * 4 + (q & 3);
            const bool rok = mt0 + rl < p.M;
            const EpiRow ri = tab[rl];
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const uint32_t e = static_cast<uint32_t>(ri.r0 + cj[j].c0) +
                                   __umul24(static_cast<uint32_t>(ri.r1), static_cast<uint32_t>(cj[j].c1)) +
                                   __umul24(static_cast<uint32_t>(ri.r2), static_cast<uint32_t>(cj[j].c2));
                const uint32_t vo = (rok && cok[j]) ? e * 4u : 0x80000000u;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(acc[i][j][q]), rc, vo, 0, 0);
            }
        }
}

__device__ __forceinline__ bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// GEMM operands always come from the library's fused workspace: 16-byte
// aligned rows whose padding past the last column is zero (the workspace is
// cleared when allocated and no kernel ever writes the padding).  Loads are
// therefore branch-free: the row index is clamped into the matrix (rows past
// the end only feed output rows that the store guard drops), the column is
// clamped into the padded row, and chunks that start past the row are zeroed.
__device__ __forceinline__ v4f load_f32x4(const float* base, int64_t ld, int r, int c, int R, int Cn) {
    (void)Cn;
    const int rr = r < R ? r : R - 1;
    const int cc = c < ld ? c : static_cast<int>(ld) - 4;
    v4f v = *reinterpret_cast<const v4f*>(base + static_cast<int64_t>(rr) * ld + cc);
    const v4f z = {0.f, 0.f, 0.f, 0.f};
    return c < ld ? v : z;
}

// Address half of load_f32x4; the caller zeroes chunks with c >= ld when it
// stores them to LDS, so nothing waits on the load right after its issue.
__device__ __forceinline__ v4f load_f32x4_raw(const float* base, int64_t ld, int r, int c, int R) {
    const int rr = r < R ? r : R - 1;
    const int cc = c < ld ? c : static_cast<int>(ld) - 4;
    return *reinterpret_cast<const v4f*>(base + static_cast<int64_t>(rr) * ld + cc);
}

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_gemm_f32(const GemmProb* __restrict__ probs, const GemmTile* __restrict__ tiles,
                                                  int n_tiles, const EpiRow* __restrict__ rows,
                                                  const EpiCol* __restrict__ cols, PtrTable bufs) {
    constexpr int KT = 16;           // K slice per stage (floats)
    constexpr int P = KT + 4;        // LDS row pitch (floats), keeps 16-byte alignment
    constexpr int WM = MT / 2, WN = NT / 2;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int AV = MT * KT / 4 / 256;   // float4 loads per thread for A
    constexpr int BV = NT * KT / 4 / 256;
    static_assert(AV >= 1 && BV >= 1, "tile too small for 256 threads");
    __shared__ __attribute__((aligned(16))) float As[2][MT * P];
    __shared__ __attribute__((aligned(16))) float Bs[2][NT * P];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, r32 = lane & 31;

    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const GemmTile tile = tiles[t];
        const GemmProb p = probs[tile.prob];
        const float* A = static_cast<const float*>(bufs.p[p.a_buf]) + p.a_off;
        const float* B = static_cast<const float*>(bufs.p[p.b_buf]) + p.b_off;
        float* C = static_cast<float*>(const_cast<void*>(bufs.p[p.c_buf])) + p.c_off;
        const int m0 = tile.tm * MT, n0 = tile.tn * NT;

        v16f acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

        v4f ra[AV], rb[BV];
        auto gload = [&](int k0) {
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const int idx = tid + i * 256;
                ra[i] = load_f32x4_raw(A, p.lda, m0 + (idx >> 2), k0 + (idx & 3) * 4, p.M);
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const int idx = tid + i * 256;
                rb[i] = load_f32x4_raw(B, p.ldb, n0 + (idx >> 2), k0 + (idx & 3) * 4, p.N);
            }
        };
        const v4f zf4 = {0.f, 0.f, 0.f, 0.f};
        auto sstore = [&](int buf, int k0) {
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const int idx = tid + i * 256;
                *reinterpret_cast<v4f*>(&As[buf][(idx >> 2) * P + (idx & 3) * 4]) = (k0 + (idx & 3) * 4 < p.lda) ? ra[i] : zf4;
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const int idx = tid + i * 256;
                *reinterpret_cast<v4f*>(&Bs[buf][(idx >> 2) * P + (idx & 3) * 4]) = (k0 + (idx & 3) * 4 < p.ldb) ? rb[i] : zf4;
            }
        };

        const int nk = (p.K + KT - 1) / KT;
        if (nk > 0) {
            gload(0);
            sstore(0, 0);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * KT);
            v4f af[FM][2], bfr[FN][2];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const float* ap = &As[cur][(wm * WM + i * 32 + r32) * P + h * 8];
                af[i][0] = *reinterpret_cast<const v4f*>(ap);
                af[i][1] = *reinterpret_cast<const v4f*>(ap + 4);
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const float* bp = &Bs[cur][(wn * WN + j * 32 + r32) * P + h * 8];
                bfr[j][0] = *reinterpret_cast<const v4f*>(bp);
                bfr[j][1] = *reinterpret_cast<const v4f*>(bp + 4);
            }
#pragma unroll
            for (int s = 0; s < 8; ++s)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[i][s >> 2][s & 3], bfr[j][s >> 2][s & 3],
                                                                         acc[i][j], 0, 0, 0);
            if (kt + 1 < nk) sstore(cur ^ 1, (kt + 1) * KT);
            __syncthreads();
        }

        // 32x32 MFMA result: lane owns column (lane & 31); register 4*i+j is
        // row 8*i + 4*(lane >> 5) + j.
        store_tile<FM, FN>(acc, p, C, rows, cols, m0 + wm * WM, n0 + wn * WN, h, r32);
    }
}

// 8 consecutive BF16 of row r from column c (as 4 dwords); same contract as
// load_f32x4 (workspace rows padded to 8 elements with zeros).
__device__ __forceinline__ u32x4 load_bf16x8(const uint16_t* base, int64_t ld, int r, int c, int R, int Cn) {
    (void)Cn;
    const int rr = r < R ? r : R - 1;
    const int cc = c < ld ? c : static_cast<int>(ld) - 8;
    u32x4 v = *reinterpret_cast<const u32x4*>(base + static_cast<int64_t>(rr) * ld + cc);
    const u32x4 z = {0u, 0u, 0u, 0u};
    return c < ld ? v : z;
}

// Address half of load_bf16x8: the caller zeroes the chunk (c >= ld) when it
// stores it to LDS, so that no instruction waits on the load right after it
// is issued.
__device__ __forceinline__ u32x4 load_bf16x8_raw(const uint16_t* base, int64_t ld, int r, int c, int R) {
    const int rr = r < R ? r : R - 1;
    const int cc = c < ld ? c : static_cast<int>(ld) - 8;
    return *reinterpret_cast<const u32x4*>(base + static_cast<int64_t>(rr) * ld + cc);
}

template <int MT, int NT>
__global__ __launch_bounds__(256) void k_gemm_bf16(const GemmProb* __restrict__ probs, const GemmTile* __restrict__ tiles,
                                                   int n_tiles, const EpiRow* __restrict__ rows,
                                                  const EpiCol* __restrict__ cols, PtrTable bufs) {
    constexpr int KT = 32;           // K slice per stage (bf16)
    constexpr int P = KT + 8;        // LDS row pitch (bf16): 80 bytes
    constexpr int WM = MT / 2, WN = NT / 2;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int AV = MT * KT / 8 / 256;   // 16-byte loads per thread for A
    constexpr int BV = NT * KT / 8 / 256;
    static_assert(AV >= 1 && BV >= 1, "tile too small for 256 threads");
    __shared__ __attribute__((aligned(16))) uint16_t As[2][MT * P];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[2][NT * P];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int h = lane >> 5, r32 = lane & 31;

    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const GemmTile tile = tiles[t];
        const GemmProb p = probs[tile.prob];
        const uint16_t* A = static_cast<const uint16_t*>(bufs.p[p.a_buf]) + p.a_off;
        const uint16_t* B = static_cast<const uint16_t*>(bufs.p[p.b_buf]) + p.b_off;
        float* C = static_cast<float*>(const_cast<void*>(bufs.p[p.c_buf])) + p.c_off;
        const int m0 = tile.tm * MT, n0 = tile.tn * NT;

        v16f acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

        u32x4 ra[AV], rb[BV];
        auto gload = [&](int k0) {
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const int idx = tid + i * 256;
                ra[i] = load_bf16x8_raw(A, p.lda, m0 + (idx >> 2), k0 + (idx & 3) * 8, p.M);
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const int idx = tid + i * 256;
                rb[i] = load_bf16x8_raw(B, p.ldb, n0 + (idx >> 2), k0 + (idx & 3) * 8, p.N);
            }
        };
        const u32x4 zu4 = {0u, 0u, 0u, 0u};
        auto sstore = [&](int buf, int k0) {
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const int idx = tid + i * 256;
                *reinterpret_cast<u32x4*>(&As[buf][(idx >> 2) * P + (idx & 3) * 8]) = (k0 + (idx & 3) * 8 < p.lda) ? ra[i] : zu4;
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const int idx = tid + i * 256;
                *reinterpret_cast<u32x4*>(&Bs[buf][(idx >> 2) * P + (idx & 3) * 8]) = (k0 + (idx & 3) * 8 < p.ldb) ? rb[i] : zu4;
            }
        };

        const int nk = (p.K + KT - 1) / KT;
        if (nk > 0) {
            gload(0);
            sstore(0, 0);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * KT);
#pragma unroll
            for (int s = 0; s < KT / 16; ++s) {
                bf16x8 af[FM], bfr[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const uint16_t* ap = &As[cur][(wm * WM + i * 32 + r32) * P + s * 16 + h * 8];
                    af[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(ap));
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const uint16_t* bp = &Bs[cur][(wn * WN + j * 32 + r32) * P + s * 16 + h * 8];
                    bfr[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(bp));
                }
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
            }
            if (kt + 1 < nk) sstore(cur ^ 1, (kt + 1) * KT);
            __syncthreads();
        }

        store_tile<FM, FN>(acc, p, C, rows, cols, m0 + wm * WM, n0 + wn * WN, h, r32);
    }
}

// Large-tile BF16 GEMM: MT x NT workgroup tile (4 waves, each (MT/2) x (NT/2)),
// K slices of KT staged through dynamic LDS in two buffers.  LDS rows are
// unpadded (KT*2 bytes = KT/8 chunks of 16 bytes) and the chunk index is
// XOR-swizzled with the Gray code of the row, so that both the 16-byte
// stores of a wave (8 chunks x 8 rows) and the MFMA operand reads (32
// consecutive rows, one chunk) hit distinct banks.
template <int CH>
__device__ __forceinline__ int swz(int r, int c) {
    return r * CH + (c ^ ((r ^ (r >> 1)) & (CH - 1)));
}

// WGM x WGN waves per workgroup, each owning an (MT/WGM) x (NT/WGN) sub-tile.
// STORE_AT: the K step after whose MFMAs the next slice is written to LDS
// (KT/16 = after all of them); storing earlier overlaps the LDS writes with
// the remaining MFMAs of the slice.
template <int MT, int NT, int KT, int WGM, int WGN, int OCC, int STORE_AT>
__global__ __launch_bounds__(64 * WGM * WGN, OCC) void k_gemm_bf16_big(const GemmProb* __restrict__ probs,
                                                                       const GemmTile* __restrict__ tiles, int n_tiles,
                                                                       const EpiRow* __restrict__ rows,
                                                                       const EpiCol* __restrict__ cols, PtrTable bufs) {
    constexpr int NTHR = 64 * WGM * WGN;
    constexpr int CH = KT / 8;
    constexpr int WM = MT / WGM, WN = NT / WGN;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int AV = MT * CH / NTHR, BV = NT * CH / NTHR;
    constexpr int S = KT / 16;
    static_assert(AV >= 1 && BV >= 1 && (CH & (CH - 1)) == 0 && FM >= 1 && FN >= 1, "bad tile");
    extern __shared__ u32x4 smem[];
    u32x4* As = smem;                  // [2][MT*CH]
    u32x4* Bs = smem + 2 * MT * CH;    // [2][NT*CH]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int h = lane >> 5, r32 = lane & 31;

    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const GemmTile tile = tiles[t];
        const GemmProb p = probs[tile.prob];
        const uint16_t* A = static_cast<const uint16_t*>(bufs.p[p.a_buf]) + p.a_off;
        const uint16_t* B = static_cast<const uint16_t*>(bufs.p[p.b_buf]) + p.b_off;
        float* C = static_cast<float*>(const_cast<void*>(bufs.p[p.c_buf])) + p.c_off;
        const int m0 = tile.tm * MT, n0 = tile.tn * NT;

        v16f acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

        u32x4 ra[AV], rb[BV];
        auto gload = [&](int k0) {
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const int idx = tid + i * NTHR;
                ra[i] = load_bf16x8_raw(A, p.lda, m0 + idx / CH, k0 + (idx % CH) * 8, p.M);
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const int idx = tid + i * NTHR;
                rb[i] = load_bf16x8_raw(B, p.ldb, n0 + idx / CH, k0 + (idx % CH) * 8, p.N);
            }
        };
        const u32x4 zero4 = {0u, 0u, 0u, 0u};
        auto sstore = [&](int buf, int k0) {
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const int idx = tid + i * NTHR;
                As[buf * MT * CH + swz<CH>(idx / CH, idx % CH)] = (k0 + (idx % CH) * 8 < p.lda) ? ra[i] : zero4;
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const int idx = tid + i * NTHR;
                Bs[buf * NT * CH + swz<CH>(idx / CH, idx % CH)] = (k0 + (idx % CH) * 8 < p.ldb) ? rb[i] : zero4;
            }
        };

        const int nk = (p.K + KT - 1) / KT;
        if (nk > 0) {
            gload(0);
            sstore(0, 0);
        }
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) gload((kt + 1) * KT);
            __builtin_amdgcn_sched_barrier(0);
            const u32x4* Ac = As + cur * MT * CH;
            const u32x4* Bc = Bs + cur * NT * CH;
            // operand fragments in two register sets: the reads for K step
            // s+1 are issued before the MFMAs of step s (the scheduling
            // barriers keep the compiler from sinking them to their use)
            u32x4 af[2][FM], bfr[2][FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) af[0][i] = Ac[swz<CH>(wm * WM + i * 32 + r32, h)];
#pragma unroll
            for (int j = 0; j < FN; ++j) bfr[0][j] = Bc[swz<CH>(wn * WN + j * 32 + r32, h)];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int cs = s & 1;
                if (s + 1 < S) {
                    const int c = 2 * (s + 1) + h;
#pragma unroll
                    for (int i = 0; i < FM; ++i) af[cs ^ 1][i] = Ac[swz<CH>(wm * WM + i * 32 + r32, c)];
#pragma unroll
                    for (int j = 0; j < FN; ++j) bfr[cs ^ 1][j] = Bc[swz<CH>(wn * WN + j * 32 + r32, c)];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[cs][i]),
                                                                             __builtin_bit_cast(bf16x8, bfr[cs][j]),
                                                                             acc[i][j], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                // the other LDS buffer was last read before the previous barrier
                if (s == STORE_AT && kt + 1 < nk) sstore(cur ^ 1, (kt + 1) * KT);
            }
            if (STORE_AT >= S && kt + 1 < nk) sstore(cur ^ 1, (kt + 1) * KT);
            __syncthreads();
        }

        store_tile<FM, FN>(acc, p, C, rows, cols, m0 + wm * WM, n0 + wn * WN, h, r32);
    }
}

template <int MT, int NT, int KT, int WGM, int WGN, int OCC, int SA>
hipError_t launch_big(const GemmProb* probs, const GemmTile* tiles, int32_t n_tiles, int32_t grid,
                      const EpiRow* rows, const EpiCol* cols, const PtrTable& bufs, hipStream_t s) {
    constexpr size_t lds = 2 * (MT + NT) * (KT / 8) * 16;
    // once per process (a thread-safe static initialisation)
    static const hipError_t configured =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_bf16_big<MT, NT, KT, WGM, WGN, OCC, SA>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (configured != hipSuccess) return configured;
    hipLaunchKernelGGL((k_gemm_bf16_big<MT, NT, KT, WGM, WGN, OCC, SA>), dim3(static_cast<unsigned>(grid)),
                       dim3(64 * WGM * WGN), lds, s, probs, tiles, n_tiles, rows, cols, bufs);
    return hipGetLastError();
}

template <int MT, int NT, int KT, int WGM, int WGN, int OCC, int SA>
int occupancy_big() {
    constexpr size_t lds = 2 * (MT + NT) * (KT / 8) * 16;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_bf16_big<MT, NT, KT, WGM, WGN, OCC, SA>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_bf16_big<MT, NT, KT, WGM, WGN, OCC, SA>,
                                                     64 * WGM * WGN, lds) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

// ---------------------------------------------------------------------------
// K6 with direct loads: operand slices go from global memory straight into
// LDS (16-byte buffer loads with the LDS bit: no staging registers, no LDS
// store instructions) through a ring of ST stages.  Iteration kt computes
// slice kt, needs slice kt + 1 in LDS (its last K step already reads the
// first fragments of the next slice, so no MFMA waits on LDS after a
// barrier) and keeps slices kt + 2 .. kt + ST - 2 in flight.
//
// A wave's load fills a 1 KB window of LDS, lane l at byte 16 l, so the row
// swizzle moves to the global side: LDS slot (r, c') receives chunk
// c' ^ f(r) of row r.  Each operand is addressed through a buffer resource
// whose base is the tile's first row and whose size ends at the tile's last
// valid row; rows past M, chunks past the padded row length and slices past
// K get an offset beyond that size, which the buffer unit's range check
// turns into zeros without accessing memory.  Requires lda, ldb multiples of
// 8 elements with zeros in columns [K, ld) (the planner's operand layouts)
// and MT * ld * 2 < 2^31 bytes (checked on the host).
// ---------------------------------------------------------------------------
constexpr int kDlMaxLd = 1 << 21;

// LDS slot of 16-byte chunk c of row r for rows of CH chunks.  The LDS serves
// a 16-byte-per-lane read 16 lanes at a time from 64 four-byte banks (256
// bytes), and a fragment read has 16 consecutive rows at one chunk: XOR-ing
// the chunk with (r / (16 / CH)) puts those rows on 16 distinct 16-byte bank
// groups.
template <int CH>
__device__ __forceinline__ int swz16(int r, int c) {
    return r * CH + (c ^ ((r / (16 / CH)) & (CH - 1)));
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
    // 0x00020000: raw (untyped) 32-bit data format, the gfx9 default
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0), static_cast<int>(bytes),
                                             0x00020000);
}

__device__ __forceinline__ void load_to_lds(__amdgpu_buffer_rsrc_t r, u32x4* lds_window, uint32_t voffset,
                                            uint32_t soffset = 0) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds_window, 16, voffset,
                                             static_cast<int>(soffset), 0, 0);
}

// s_waitcnt immediate that waits until at most n vector memory operations of
// this wave are outstanding (expcnt and lgkmcnt left unconstrained)
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | 0x0F70; }

// OPT bit 0: raise the wave's issue priority while it issues MFMAs; bit 1:
// interleave the next step's fragment reads with the MFMAs one by one; bit
// 3: one barrier per two K slices (five stages); bit 5: a slice that lies
// wholly inside the padded rows is loaded with the per-lane offsets of the
// tile's first slice and the slice's K offset as a scalar offset (no
// per-load vector arithmetic); bit 6: the same slices with the K offset
// added to each lane's offset (one add per load, no range tests).
template <int MT, int NT, int KT, int WGM, int WGN, int ST, int OPT>
__global__ __launch_bounds__(64 * WGM * WGN, 1) void k_gemm_bf16_dl(const GemmProb* __restrict__ probs,
                                                                    const GemmTile* __restrict__ tiles, int n_tiles,
                                                                    const EpiRow* __restrict__ rows,
                                                                    const EpiCol* __restrict__ cols, PtrTable bufs) {
    constexpr int NTHR = 64 * WGM * WGN;
    constexpr int CH = KT / 8;
    constexpr int WM = MT / WGM, WN = NT / WGN;
    constexpr int FM = WM / 32, FN = WN / 32;
    constexpr int AV = MT * CH / NTHR, BV = NT * CH / NTHR;
    constexpr int SA = MT * CH, SB = NT * CH;
    constexpr int S = KT / 16;
    static_assert(AV >= 1 && BV >= 1 && AV * NTHR == SA && BV * NTHR == SB && (CH & (CH - 1)) == 0 && CH <= 16 &&
                      ST >= 3 && S % 2 == 0,
                  "bad tile");
    extern __shared__ u32x4 smem[];
    u32x4* As = smem;            // [ST][SA]
    u32x4* Bs = smem + ST * SA;  // [ST][SB]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const int h = lane >> 5, r32 = lane & 31;

    // the LDS slot of each of this thread's loads, and the row and column
    // (in elements, within a slice) whose chunk it receives
    int a_row[AV], a_col[AV], b_row[BV], b_col[BV];
#pragma unroll
    for (int i = 0; i < AV; ++i) {
        const int p = tid + i * NTHR, r = p / CH;
        a_row[i] = r;
        a_col[i] = ((p % CH) ^ ((r / (16 / CH)) & (CH - 1))) * 8;
    }
#pragma unroll
    for (int i = 0; i < BV; ++i) {
        const int p = tid + i * NTHR, r = p / CH;
        b_row[i] = r;
        b_col[i] = ((p % CH) ^ ((r / (16 / CH)) & (CH - 1))) * 8;
    }

    for (int t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const GemmTile tile = tiles[t];
        const GemmProb p = probs[tile.prob];
        const uint16_t* A = static_cast<const uint16_t*>(bufs.p[p.a_buf]) + p.a_off;
        const uint16_t* B = static_cast<const uint16_t*>(bufs.p[p.b_buf]) + p.b_off;
        float* C = static_cast<float*>(const_cast<void*>(bufs.p[p.c_buf])) + p.c_off;
        const int m0 = tile.tm * MT, n0 = tile.tn * NT;

        // the previous tile's loads and stores are complete and every wave is
        // done reading its stages before this tile's loads overwrite them
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_sched_barrier(0);

        const int a_rows = min(MT, p.M - m0), b_rows = min(NT, p.N - n0);
        const __amdgpu_buffer_rsrc_t ra =
            make_rsrc(A + static_cast<int64_t>(m0) * p.lda, static_cast<uint32_t>(a_rows) * p.lda * 2u);
        const __amdgpu_buffer_rsrc_t rb =
            make_rsrc(B + static_cast<int64_t>(n0) * p.ldb, static_cast<uint32_t>(b_rows) * p.ldb * 2u);
        uint32_t a_vo[AV], b_vo[BV];
#pragma unroll
        for (int i = 0; i < AV; ++i) a_vo[i] = (static_cast<uint32_t>(a_row[i]) * p.lda + a_col[i]) * 2u;
#pragma unroll
        for (int i = 0; i < BV; ++i) b_vo[i] = (static_cast<uint32_t>(b_row[i]) * p.ldb + b_col[i]) * 2u;

        const int nk = (p.K + KT - 1) / KT;
        // slices at or past nk are issued too (all lanes out of range, so
        // they only write zeros to a stage nobody reads): that keeps the
        // number of loads in flight, and so the wait below, the same for
        // every slice
        auto issue = [&](int kt, int stage) {
            const int k0 = kt * KT;
            const bool live = kt < nk;
            if constexpr ((OPT & 32) != 0) {
                // uniform: every chunk of the slice is inside the padded rows
                if (live && k0 + KT <= p.lda && k0 + KT <= p.ldb) {
                    const uint32_t so = 2u * static_cast<uint32_t>(k0);
#pragma unroll
                    for (int i = 0; i < AV; ++i) load_to_lds(ra, As + stage * SA + i * NTHR + wave * 64, a_vo[i], so);
#pragma unroll
                    for (int i = 0; i < BV; ++i) load_to_lds(rb, Bs + stage * SB + i * NTHR + wave * 64, b_vo[i], so);
                    return;
                }
            }
            if constexpr ((OPT & 64) != 0) {
                // the same test, the K offset added to each lane's offset
                if (live && k0 + KT <= p.lda && k0 + KT <= p.ldb) {
                    const uint32_t so = 2u * static_cast<uint32_t>(k0);
#pragma unroll
                    for (int i = 0; i < AV; ++i) load_to_lds(ra, As + stage * SA + i * NTHR + wave * 64, a_vo[i] + so);
#pragma unroll
                    for (int i = 0; i < BV; ++i) load_to_lds(rb, Bs + stage * SB + i * NTHR + wave * 64, b_vo[i] + so);
                    return;
                }
            }
#pragma unroll
            for (int i = 0; i < AV; ++i) {
                const uint32_t vo = (live && k0 + a_col[i] < p.lda) ? a_vo[i] + 2u * k0 : 0x80000000u;
                load_to_lds(ra, As + stage * SA + i * NTHR + wave * 64, vo);
            }
#pragma unroll
            for (int i = 0; i < BV; ++i) {
                const uint32_t vo = (live && k0 + b_col[i] < p.ldb) ? b_vo[i] + 2u * k0 : 0x80000000u;
                load_to_lds(rb, Bs + stage * SB + i * NTHR + wave * 64, vo);
            }
        };

        v16f acc[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int q = 0; q < 16; ++q) acc[i][j][q] = 0.f;

        // fragments of one K step (16) of the slice in stage st
        u32x4 af[2][FM], bfr[2][FN];
        auto frags = [&](int st, int step, int set) {
            const u32x4* Ac = As + st * SA;
            const u32x4* Bc = Bs + st * SB;
            const int c = 2 * step + h;
#pragma unroll
            for (int i = 0; i < FM; ++i) af[set][i] = Ac[swz16<CH>(wm * WM + i * 32 + r32, c)];
#pragma unroll
            for (int j = 0; j < FN; ++j) bfr[set][j] = Bc[swz16<CH>(wn * WN + j * 32 + r32, c)];
        };

        // the MFMAs of the slice in stage sr; its last step reads the first
        // fragments of the slice in stage sn
        auto slice = [&](int sr, int sn) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int cs = s & 1;
                // the last step fetches the first fragments of the next slice,
                // so the MFMAs never wait on LDS after the barrier
                const int st = s + 1 < S ? sr : sn, step = s + 1 < S ? s + 1 : 0;
                if constexpr ((OPT & 2) == 0) {
                    frags(st, step, cs ^ 1);
                    __builtin_amdgcn_sched_barrier(0);
                }
                if constexpr ((OPT & 1) != 0) __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) {
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, af[cs][i]),
                                                                             __builtin_bit_cast(bf16x8, bfr[cs][j]),
                                                                             acc[i][j], 0, 0, 0);
                        if constexpr ((OPT & 2) != 0) {
                            // after MFMA number f, read fragment f of the next step
                            // (B fragments first: the next step opens with A0 x B0)
                            const int f = i * FN + j;
                            const u32x4* Ac = As + st * SA;
                            const u32x4* Bc = Bs + st * SB;
                            const int c = 2 * step + h;
                            if (f < FN) bfr[cs ^ 1][f] = Bc[swz16<CH>(wn * WN + f * 32 + r32, c)];
                            else if (f < FM + FN)
                                af[cs ^ 1][f - FN] = Ac[swz16<CH>(wm * WM + (f - FN) * 32 + r32, c)];
                            __builtin_amdgcn_sched_barrier(0);
                        }
                    }
                if constexpr ((OPT & 1) != 0) __builtin_amdgcn_s_setprio(0);
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        auto wrap = [](int x) { return x >= ST ? x - ST : x; };

        if constexpr ((OPT & 8) != 0) {
            // one barrier per two slices: slices kt .. kt + 2 are in LDS when
            // the pair (kt, kt + 1) starts, kt + 3 and kt + 4 go into the
            // stages the previous pair used (five stages)
            static_assert(ST == 5, "paired slices need five stages");
#pragma unroll
            for (int s = 0; s < 3; ++s) issue(s, s);
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
            frags(0, 0, 0);
            int sr = 0;   // stage of slice kt
            for (int kt = 0; kt < nk; kt += 2) {
                // every load issued so far (slices up to kt + 2) has landed
                // for this wave; after the barrier for every wave, and every
                // wave is done with slices kt - 2 and kt - 1
                __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_sched_barrier(0);
                const int s1 = wrap(sr + 1), s2 = wrap(sr + 2), s3 = wrap(sr + 3), s4 = wrap(sr + 4);
                issue(kt + 3, s3);
                issue(kt + 4, s4);
                __builtin_amdgcn_sched_barrier(0);
                slice(sr, s1);
                if (kt + 1 < nk) slice(s1, s2);
                sr = s2;
            }
        } else {
#pragma unroll
            for (int s = 0; s < ST - 1; ++s) issue(s, s);
            // slice 0 visible to every wave
            __builtin_amdgcn_s_waitcnt(vmcnt_imm((ST - 2) * (AV + BV)));
            __builtin_amdgcn_s_barrier();
            __builtin_amdgcn_sched_barrier(0);
            frags(0, 0, 0);
            int sr = 0, sw = ST - 1;
            for (int kt = 0; kt < nk; ++kt) {
                // slices kt and kt + 1 have landed for this wave; after the
                // barrier for every wave, and every wave is done with iteration
                // kt - 1, so stage sw (slice kt - 1) is free
                __builtin_amdgcn_s_waitcnt(vmcnt_imm((ST - 3) * (AV + BV)));
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_sched_barrier(0);
                issue(kt + ST - 1, sw);
                __builtin_amdgcn_sched_barrier(0);
                const int sn = wrap(sr + 1);
                slice(sr, sn);
                sr = sn;
                sw = wrap(sw + 1);
            }
        }

        if (p.indirect) {
            // the stages are free once the trailing (all zero) slice loads
            // have landed and every wave is past its last fragment reads
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
            __builtin_amdgcn_s_barrier();
            EpiRow* tab = reinterpret_cast<EpiRow*>(smem);
            for (int r = tid; r < MT; r += NTHR) tab[r] = rows[p.ri_off + min(m0 + r, p.M - 1)];
            __syncthreads();
            store_tile_tab<FM, FN>(acc, p, C, tab, cols, m0, wm * WM, n0 + wn * WN, h, r32);
        } else {
            store_tile<FM, FN>(acc, p, C, rows, cols, m0 + wm * WM, n0 + wn * WN, h, r32);
        }
    }
    // no load may still be writing LDS when the workgroup ends
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
}

template <int MT, int NT, int KT, int ST>
constexpr size_t dl_lds_bytes() {
    return static_cast<size_t>(ST) * (MT + NT) * (KT / 8) * 16;
}

template <int MT, int NT, int KT, int WGM, int WGN, int ST, int OPT>
hipError_t launch_dl(const GemmProb* probs, const GemmTile* tiles, int32_t n_tiles, int32_t grid, const EpiRow* rows,
                     const EpiCol* cols, const PtrTable& bufs, hipStream_t s) {
    constexpr size_t lds = dl_lds_bytes<MT, NT, KT, ST>();
    // once per process (a thread-safe static initialisation)
    static const hipError_t configured =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_bf16_dl<MT, NT, KT, WGM, WGN, ST, OPT>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (configured != hipSuccess) return configured;
    hipLaunchKernelGGL((k_gemm_bf16_dl<MT, NT, KT, WGM, WGN, ST, OPT>), dim3(static_cast<unsigned>(grid)),
                       dim3(64 * WGM * WGN), lds, s, probs, tiles, n_tiles, rows, cols, bufs);
    return hipGetLastError();
}

template <int MT, int NT, int KT, int WGM, int WGN, int ST, int OPT>
int occupancy_dl() {
    constexpr size_t lds = dl_lds_bytes<MT, NT, KT, ST>();
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_bf16_dl<MT, NT, KT, WGM, WGN, ST, OPT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_bf16_dl<MT, NT, KT, WGM, WGN, ST, OPT>, 64 * WGM * WGN,
                                                     lds) != hipSuccess)
        n = 1;
    return n > 0 ? n : 1;
}

// direct-load variants: (variant, MT, NT, KT, WGM, WGN, stages)
#define SYM_BF16_DL_VARIANTS(X)        \
    X(9, 256, 256, 32, 2, 4, 4, 0)     \
    X(10, 256, 256, 32, 2, 4, 5, 0)    \
    X(11, 256, 256, 32, 2, 2, 5, 0)    \
    X(12, 256, 256, 32, 2, 4, 5, 1)    \
    X(13, 256, 256, 32, 2, 4, 5, 2)    \
    X(14, 256, 256, 32, 2, 4, 5, 3)    \
    X(15, 256, 256, 32, 2, 2, 5, 1)    \
    X(16, 256, 256, 32, 2, 4, 5, 10)   \
    X(17, 256, 256, 32, 2, 4, 5, 42)   \
    X(18, 256, 256, 32, 2, 4, 5, 67)

bool gemm_variant_direct(int compute, int variant) { return compute == 1 && variant >= 9 && variant <= 18; }

int gemm_direct_max_ld() { return kDlMaxLd; }

// BF16 variants: v0-v2 and v5-v8 are k_gemm_bf16_big instances (tile, wave
// grid, residency, LDS-store placement); v3, v4 the K=32 padded-LDS kernel;
// v9-v18 k_gemm_bf16_dl.
#define SYM_BF16_BIG_VARIANTS(X)              \
    X(0, 256, 256, 64, 2, 2, 1, 4)            \
    X(1, 256, 128, 64, 2, 2, 1, 4)            \
    X(2, 128, 128, 64, 2, 2, 2, 4)            \
    X(5, 256, 256, 64, 2, 4, 2, 4)            \
    X(6, 256, 128, 64, 4, 2, 2, 1)            \
    X(7, 128, 128, 64, 2, 2, 2, 1)            \
    X(8, 256, 128, 64, 4, 2, 2, 4)

namespace {
const GemmVariant kF32Variants[] = {{128, 128, "k_gemm_f32 128x128"},
                                    {64, 64, "k_gemm_f32 64x64"},
                                    {128, 64, "k_gemm_f32 128x64"},
                                    {256, 128, "k_gemm_f32 256x128"}};
const GemmVariant kBF16Variants[] = {{256, 256, "k_gemm_bf16_big 256x256 k64 4w"},
                                     {256, 128, "k_gemm_bf16_big 256x128 k64 4w"},
                                     {128, 128, "k_gemm_bf16_big 128x128 k64 4w occ2"},
                                     {128, 128, "k_gemm_bf16 128x128 k32"},
                                     {64, 64, "k_gemm_bf16 64x64 k32"},
                                     {256, 256, "k_gemm_bf16_big 256x256 k64 8w"},
                                     {256, 128, "k_gemm_bf16_big 256x128 k64 8w early-store"},
                                     {128, 128, "k_gemm_bf16_big 128x128 k64 4w early-store"},
                                     {256, 128, "k_gemm_bf16_big 256x128 k64 8w"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 4-stage"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 4w 5-stage"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage prio"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage interleaved"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage prio interleaved"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 4w 5-stage prio"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage interleaved paired"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage interleaved paired soffset"},
                                     {256, 256, "k_gemm_bf16_dl 256x256 k32 8w 5-stage prio interleaved koff"}};
}  // namespace

int gemm_num_variants(int compute) { return compute == 0 ? 4 : 19; }
GemmVariant gemm_variant(int compute, int v) { return compute == 0 ? kF32Variants[v] : kBF16Variants[v]; }
// FP32: 128x128 by default; 256x128 (two waves per SIMD, each 128 x 64)
// ran the FP32 batch 4 % faster and config 4's smaller sectors 11 % slower,
// so it is left to the autotuner.
// Defaults from measurements on MI355X.  256x256 tiles (operand re-reads
// beyond L2 fall with the tile size: 128x128 ran the 64-member batch at 377
// TFLOP/s) with 8 waves, two per SIMD, fed by direct loads through a
// five-stage LDS ring: 990 to 1060 TFLOP/s on the batch and about 1190 on
// one 8192^3 product, against 901 on the batch for the register-staged
// 256x256 kernel on the same GPU.  With one barrier per two K slices and
// the fragment reads interleaved with the MFMAs (variant 16) the batch ran
// at 1031 to 1041 TFLOP/s in five alternating rounds, where the same
// kernel with a barrier per slice ranged from 979 to 1055 (median 995).
// Loading the slices that lie wholly inside the padded rows with a scalar K
// offset (variant 17: no per-load vector arithmetic) took the batch from
// 50.97 to 50.07 ms (median of six alternating rounds, bitwise equal), but
// ran the GEMM of the literal-dimension prefix (sectors up to about 26000)
// at 708 to 767 ms against 590 to 654 for the per-lane-offset kernels.  The
// default is the interleaved kernel with raised MFMA priority and a barrier
// per slice (variant 14): on one MI355X, alternating, it ran the batch at
// 54.0 ms against 55.1 (17), 55.7 (16) and 56.3 (paired with priority),
// and the prefix at 590 ms against 625 and 652.  The same kernel with the
// whole-slice loads' K offset added per lane (variant 18) ran the batch at
// 51.1 against 53.3 ms on another MI355X but the prefix at 615 against 591
// ms (the paired kernel with that load path: 774 ms).  The ranking of the
// 256x256 variants moves from one MI355X to another, which is what the
// autotuner is for.
int gemm_default_variant(int compute) { return compute == 0 ? 0 : 14; }
int gemm_default_variant_wide(int compute) { return compute == 0 ? 0 : 5; }

const char* gemm_variant_kernel(int compute, int variant) {
    if (compute == 0) {
        static const char* const f32[] = {"k_gemm_f32<128, 128>", "k_gemm_f32<64, 64>", "k_gemm_f32<128, 64>",
                                          "k_gemm_f32<256, 128>"};
        return variant >= 0 && variant < 4 ? f32[variant] : "";
    }
    switch (variant) {
#define SYM_SIG_BIG(V, MT, NT, KT, WGM, WGN, OCC, SA) \
    case V: return "k_gemm_bf16_big<" #MT ", " #NT ", " #KT ", " #WGM ", " #WGN ", " #OCC ", " #SA ">";
        SYM_BF16_BIG_VARIANTS(SYM_SIG_BIG)
#undef SYM_SIG_BIG
#define SYM_SIG_DL(V, MT, NT, KT, WGM, WGN, ST, OPT) \
    case V: return "k_gemm_bf16_dl<" #MT ", " #NT ", " #KT ", " #WGM ", " #WGN ", " #ST ", " #OPT ">";
        SYM_BF16_DL_VARIANTS(SYM_SIG_DL)
#undef SYM_SIG_DL
        case 3: return "k_gemm_bf16<128, 128>";
        case 4: return "k_gemm_bf16<64, 64>";
        default: return "";
    }
}

int gemm_blocks_per_cu(int compute, int variant) {
    int n = 0;
    hipError_t e = hipSuccess;
    if (compute == 0) {
        switch (variant) {
            case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_f32<64, 64>, 256, 0); break;
            case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_f32<128, 64>, 256, 0); break;
            case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_f32<256, 128>, 256, 0); break;
            default: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_f32<128, 128>, 256, 0); break;
        }
    } else {
        switch (variant) {
#define SYM_OCC_CASE(V, MT, NT, KT, WGM, WGN, OCC, SA) \
    case V: return occupancy_big<MT, NT, KT, WGM, WGN, OCC, SA>();
            SYM_BF16_BIG_VARIANTS(SYM_OCC_CASE)
#undef SYM_OCC_CASE
#define SYM_OCC_DL_CASE(V, MT, NT, KT, WGM, WGN, ST, OPT) \
    case V: return occupancy_dl<MT, NT, KT, WGM, WGN, ST, OPT>();
            SYM_BF16_DL_VARIANTS(SYM_OCC_DL_CASE)
#undef SYM_OCC_DL_CASE
            case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_bf16<128, 128>, 256, 0); break;
            case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm_bf16<64, 64>, 256, 0); break;
            default: break;
        }
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_gemm(int compute, int variant, const GemmProb* probs, const GemmTile* tiles, int32_t n_tiles,
                       int32_t grid, const EpiRow* rows, const EpiCol* cols, const PtrTable& bufs, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    dim3 g(static_cast<unsigned>(grid)), b(256);
    if (compute == 0) {
        switch (variant) {
            case 1: hipLaunchKernelGGL((k_gemm_f32<64, 64>), g, b, 0, s, probs, tiles, n_tiles, rows, cols, bufs); break;
            case 2: hipLaunchKernelGGL((k_gemm_f32<128, 64>), g, b, 0, s, probs, tiles, n_tiles, rows, cols, bufs); break;
            case 3: hipLaunchKernelGGL((k_gemm_f32<256, 128>), g, b, 0, s, probs, tiles, n_tiles, rows, cols, bufs); break;
            default: hipLaunchKernelGGL((k_gemm_f32<128, 128>), g, b, 0, s, probs, tiles, n_tiles, rows, cols, bufs); break;
        }
        return hipGetLastError();
    }
    switch (variant) {
#define SYM_LAUNCH_CASE(V, MT, NT, KT, WGM, WGN, OCC, SA) \
    case V: return launch_big<MT, NT, KT, WGM, WGN, OCC, SA>(probs, tiles, n_tiles, grid, rows, cols, bufs, s);
        SYM_BF16_BIG_VARIANTS(SYM_LAUNCH_CASE)
#undef SYM_LAUNCH_CASE
#define SYM_LAUNCH_DL_CASE(V, MT, NT, KT, WGM, WGN, ST, OPT) \
    case V: return launch_dl<MT, NT, KT, WGM, WGN, ST, OPT>(probs, tiles, n_tiles, grid, rows, cols, bufs, s);
        SYM_BF16_DL_VARIANTS(SYM_LAUNCH_DL_CASE)
#undef SYM_LAUNCH_DL_CASE
        case 3: hipLaunchKernelGGL((k_gemm_bf16<128, 128>), g, b, 0, s, probs, tiles, n_tiles, rows, cols, bufs); break;
        case 4: hipLaunchKernelGGL((k_gemm_bf16<64, 64>), g, b, 0, s, probs, tiles, n_tiles, rows, cols, bufs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block-wise SVD (eq:svd0, eq:svd1): every sector matrix is factorised on its
// own, in FP64, by one-sided Jacobi (Hestenes): the k vectors are
// orthogonalised pairwise by plane rotations, the same rotations accumulate
// in Q; at convergence the vector norms are the singular values, the
// normalised vectors one set of singular vectors and Q the other.  A sweep
// is a sequence of rounds of the round-robin (circle) schedule over blocks of
// vectors; a round of every sector runs at once (one workgroup per pair of
// blocks, disjoint pairs, two launches per round), so launch boundaries
// order the rounds and the whole GPU works on them.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double as_f64(T x);
template <>
__device__ __forceinline__ double as_f64<float>(float x) { return static_cast<double>(x); }
template <>
__device__ __forceinline__ double as_f64<uint16_t>(uint16_t x) { return static_cast<double>(bf16_to_f32(x)); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// player at slot j of round r in the circle schedule over kp (even) players
__device__ __forceinline__ int rr_player(int j, int r, int kp) { return j == 0 ? 0 : 1 + (j - 1 + r) % (kp - 1); }

// vectors in FP64 (rows of the sector matrix, or its columns) and Q = I
// and each sector's squared Frobenius norm (scale[s], cleared beforehand; the
// rotations keep it)
template <typename Ti>
__global__ __launch_bounds__(256) void k_svd_load(const Ti* __restrict__ src, const SvdProb* __restrict__ probs,
                                                   double* __restrict__ Wg, double* __restrict__ Qg,
                                                   double* __restrict__ scale) {
    __shared__ double part[4];
    const SvdProb p = probs[blockIdx.y];
    const int64_t nw = static_cast<int64_t>(p.k) * p.L, nq = static_cast<int64_t>(p.k) * p.k;
    double ss = 0.0;
    for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < nw + nq; idx += static_cast<int64_t>(gridDim.x) * 256) {
        if (idx < nw) {
            const int j = static_cast<int>(idx / p.L), x = static_cast<int>(idx - static_cast<int64_t>(j) * p.L);
            const int64_t e =
                p.rows_are_vectors ? static_cast<int64_t>(j) * p.ld + x : static_cast<int64_t>(x) * p.ld + j;
            double v = as_f64(src[p.src_off + e]);
            // eigen mode: the symmetric part of the square sector matrix
            if (p.sym) v = 0.5 * (v + as_f64(src[p.src_off + static_cast<int64_t>(x) * p.ld + j]));
            Wg[p.w_off + idx] = v;
            ss = fma(v, v, ss);
        } else {
            const int64_t q = idx - nw;
            Qg[p.q_off + q] = (q / p.k == q % p.k) ? 1.0 : 0.0;
        }
    }
    ss = wave_sum(ss);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(&scale[blockIdx.y], part[0] + part[1] + part[2] + part[3]);
}

// Eigen mode: the symmetric part S of a sector becomes S + c I with c its
// Frobenius norm (1 when S = 0), which is symmetric positive definite (the
// spectral norm is at most c), so its singular value decomposition is its
// eigen-decomposition: U = V are the eigenvectors of S and each singular
// value is an eigenvalue of S plus c.  One workgroup per sector.
__global__ __launch_bounds__(256) void k_eig_shift(const SvdProb* __restrict__ probs, double* __restrict__ Wg,
                                                   const double* __restrict__ scale, double* __restrict__ shift) {
    const SvdProb p = probs[blockIdx.x];
    const double fro = sqrt(scale[blockIdx.x]);
    const double c = fro > 0.0 ? fro : 1.0;
    for (int j = threadIdx.x; j < p.k; j += 256) Wg[p.w_off + static_cast<int64_t>(j) * p.L + j] += c;
    if (threadIdx.x == 0) shift[blockIdx.x] = c;
}

// One round of block Jacobi over every sector: the vectors of a sector form blocks
// of kSvdBlock; a workgroup takes one pair of blocks (2b vectors, round-robin
// schedule over the blocks) and
//   1. forms their Gram matrix G (2b x 2b) in FP64, streaming the vectors
//      through LDS in chunks of 4096 / 2b entries (16 loads in flight per
//      thread);
//   2. makes one sweep of cyclic two-sided Jacobi on G in LDS (b disjoint
//      plane rotations per step, the same rotation as the one-sided
//      method's, accumulated in V);
//   3. replaces the 2b vectors, and their 2b rows of Q, by their products
//      with V.
// The vectors are read twice and written once per round instead of once per
// scalar round, and a sweep has nb - 1 rounds instead of k - 1.  The sweep
// counts as converged for the pair when the Jacobi sweep on G finds
// every off-diagonal entry below sqrt(L) 2^-53 of the geometric mean of its diagonal
// entries (the one-sided method's test).  Vectors past k are zero and are
// never written.
// A round is two launches over (block pair, slice), with kSvdSlices slices of
// the vector entries per pair: PHASE 0 writes each slice's partial Gram
// matrix to Gpart; PHASE 1 sums the partials in a fixed order (every slice
// gets the same G, so results do not depend on scheduling), makes the small
// Jacobi sweep and updates its slice of the vectors and of Q.  Two launches
// measured faster than one launch doing both phases (or more inner sweeps
// per round) on the largest SVD workload.  Blocks of 16 vectors halve the
// rounds of a sweep against blocks of 8 for the same bytes per round
// (config 4's SVD: 0.52 against 0.65 s); a round then does four times the
// arithmetic per entry, which the update keeps in registers by reading each
// row of V from LDS once per chunk (holding all of V, 32 x 8 doubles per
// thread, spilled).  With 16-vector blocks the largest workload has about
// 450 block pairs per round, under two workgroups per CU: two slices per
// pair measured 223 us per round against 250 us with one and 249 us with
// four.
template <int PHASE>
__global__ __launch_bounds__(256) void k_svd_bround(const SvdProb* __restrict__ probs, int n_probs,
                                                     const int32_t* __restrict__ pair_start, int r,
                                                     double* __restrict__ Wg, double* __restrict__ Qg,
                                                     const double* __restrict__ scale, double* __restrict__ Gpart,
                                                     int32_t* __restrict__ rotated, int32_t* __restrict__ lastrot,
                                                     int gidx, int R) {
    constexpr int B = kSvdBlock, B2 = 2 * B, NP = B2 / 2;
    constexpr int XC = 4096 / B2;              // chunk entries: 16 loads per thread
    constexpr int NB4 = B2 / 4;                // 4 x 4 blocks of G per row
    constexpr int LPB = 256 / (NB4 * NB4);     // lanes that share one block of G
    constexpr int JW = B2 / 4;                 // new vectors per wave in the update
    static_assert((B2 == 16 || B2 == 32) && LPB >= 1 && (LPB & (LPB - 1)) == 0 && XC % LPB == 0 && XC % 64 == 0,
                  "thread roles below assume 16 or 32 vectors per block pair");
    __shared__ double T[B2][XC + 1];
    __shared__ double G[B2][B2 + 1];
    __shared__ double V[B2][B2 + 1];
    __shared__ double cs[NP][2];
    __shared__ int s_rot, s_any;
    const int tid = static_cast<int>(threadIdx.x);
    const int pid = static_cast<int>(blockIdx.x), slice = static_cast<int>(blockIdx.y);
    constexpr int S = kSvdSlices;
    if (pid >= pair_start[n_probs]) return;
    int lo = 0, hi = n_probs - 1;   // sector of this block pair
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pair_start[mid] <= pid) lo = mid;
        else hi = mid - 1;
    }
    const SvdProb p = probs[lo];
    const int k = p.k, L = p.L;
    const int nb = (k + B - 1) / B, nbp = nb + (nb & 1);
    if (k < 2 || r >= nbp - 1) return;
    const int pi = pid - pair_start[lo];
    const int P = rr_player(pi, r, nbp), Qb = rr_player(nbp - 1 - pi, r, nbp);
    // the pair met R rounds ago (same round of the previous sweep) and was
    // left alone then; if neither block has rotated since, its Gram matrix
    // is unchanged and the pair would again be left alone: skip it (both
    // launches take the same decision, the rotation launch records the
    // round in which a block last rotated)
    int32_t* lr = lastrot + 2 * pair_start[lo];
    const int prev = gidx - R;
    if (prev >= 0 && lr[P] < prev && lr[Qb] < prev) return;
    auto col = [&](int i) { return i < B ? P * B + i : Qb * B + (i - B); };
    double* W = Wg + p.w_off;
    double* Qm = Qg + p.q_off;
    // pairs whose inner product is below 1e-30 of the sector's squared norm
    // are left alone: rotating them moves no singular value by more than
    // 1e-15 of the largest, and vectors that tend to zero (rank deficiency)
    // would otherwise keep rotating on rounding noise
    const double floor_abs = 1e-30 * scale[lo];
    // a pair counts as orthogonal once |g_pq| <= sqrt(L) u sqrt(g_pp g_qq)
    // (u = 2^-53, the unit roundoff): the rounding error of an inner product
    // of length L grows like sqrt(L) u, the one-sided Jacobi stopping rule of
    // Drmac and Veselic (the threshold LAPACK's dgesvj uses)
    const double tol_rel = sqrt(static_cast<double>(L)) * 1.1102230246251565e-16;
    // this slice's entries of the vectors (length L) and of the rows of Q
    // (length k), whole chunks each
    auto span = [&](int len, int& a, int& b) {
        const int per = ((len + S - 1) / S + XC - 1) / XC * XC;
        a = min(len, slice * per);
        b = min(len, a + per);
    };
    double* Gp = Gpart + static_cast<int64_t>(pid) * S * (B2 * B2);

    // a chunk: NL loads per thread, all issued before the first LDS write
    constexpr int NL = B2 * XC / 256;
    auto stage = [&](const double* base, int Lx, int x0, int xend) {
        double v[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int idx = tid + 256 * u, i = idx / XC, xx = idx - i * XC;
            const int c = col(i), x = x0 + xx;
            v[u] = (c < k && x < xend) ? base[static_cast<int64_t>(c) * Lx + x] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int idx = tid + 256 * u, i = idx / XC, xx = idx - i * XC;
            T[i][xx] = v[u];
        }
    };
    if constexpr (PHASE == 0) {
        // 1. Gram matrix: thread (blk, xl) sums a 4 x 4 block of G over the chunk
        //    entries xl, xl + LPB, xl + 2 LPB, ...; the LPB partial sums of a block
        //    sit in LPB consecutive lanes
        const int blk = tid / LPB, xl = tid % LPB, I4 = (blk / NB4) * 4, J4 = (blk % NB4) * 4;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        int xa, xb;
        span(L, xa, xb);
        for (int x0 = xa; x0 < xb; x0 += XC) {
            stage(W, L, x0, xb);
            __syncthreads();
#pragma unroll 4
            for (int u = 0; u < XC / LPB; ++u) {
                const int xx = xl + LPB * u;
                double va[4], vb[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) va[a] = T[I4 + a][xx];
#pragma unroll
                for (int b = 0; b < 4; ++b) vb[b] = T[J4 + b][xx];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = fma(va[a], vb[b], acc[a][b]);
            }
            __syncthreads();
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double v = acc[a][b];
#pragma unroll
                for (int o = LPB / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
                acc[a][b] = v;
            }
        if (xl == 0)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) Gp[slice * (B2 * B2) + (I4 + a) * B2 + J4 + b] = acc[a][b];
        return;
    }
    for (int idx = tid; idx < B2 * B2; idx += 256) {
        double g = 0.0;
        for (int sl = 0; sl < S; ++sl) g += Gp[sl * (B2 * B2) + idx];
        G[idx / B2][idx % B2] = g;
        V[idx / B2][idx % B2] = (idx / B2 == idx % B2) ? 1.0 : 0.0;
    }
    if (tid == 0) s_any = 0;
    __syncthreads();

    // 2. cyclic Jacobi on G: step r2 rotates the NP disjoint pairs of the
    //    circle schedule over the 16 indices.  With the rotations R_m of the
    //    pairs, every 2 x 2 block (m1, m2) of G becomes R_m1^T G R_m2 and the
    //    columns of V of pair m become V R_m: one phase, disjoint entries.
    //    One sweep per round: the outer sweeps finish the job.
    constexpr int kInner = 1;
    for (int sweep = 0; sweep < kInner; ++sweep) {
        if (tid == 0) s_rot = 0;
        __syncthreads();
        for (int r2 = 0; r2 < B2 - 1; ++r2) {
            if (tid < NP) {
                const int a = rr_player(tid, r2, B2), b = rr_player(B2 - 1 - tid, r2, B2);
                const int pp = a < b ? a : b, qq = a < b ? b : a;
                const double al = G[pp][pp], be = G[qq][qq], ga = G[pp][qq];
                double c = 1.0, sn = 0.0;
                if (ga != 0.0 && fabs(ga) > tol_rel * sqrt(fabs(al * be)) && fabs(ga) > floor_abs) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    c = 1.0 / sqrt(1.0 + t * t);
                    sn = c * t;
                    s_rot = 1;
                }
                cs[tid][0] = c;
                cs[tid][1] = sn;
            }
            __syncthreads();
            for (int it = tid; it < NP * NP + B2 * NP; it += 256) {
              if (it < NP * NP) {
                const int m1 = it / NP, m2 = it - m1 * NP;
                const int a1 = rr_player(m1, r2, B2), b1 = rr_player(B2 - 1 - m1, r2, B2);
                const int a2 = rr_player(m2, r2, B2), b2 = rr_player(B2 - 1 - m2, r2, B2);
                const int p1 = a1 < b1 ? a1 : b1, q1 = a1 < b1 ? b1 : a1;
                const int p2 = a2 < b2 ? a2 : b2, q2 = a2 < b2 ? b2 : a2;
                const double c1 = cs[m1][0], s1 = cs[m1][1], c2 = cs[m2][0], s2 = cs[m2][1];
                const double g11 = G[p1][p2], g12 = G[p1][q2], g21 = G[q1][p2], g22 = G[q1][q2];
                const double t11 = c1 * g11 - s1 * g21, t12 = c1 * g12 - s1 * g22;   // R1^T G
                const double t21 = s1 * g11 + c1 * g21, t22 = s1 * g12 + c1 * g22;
                G[p1][p2] = c2 * t11 - s2 * t12;                                      // (R1^T G) R2
                G[p1][q2] = s2 * t11 + c2 * t12;
                G[q1][p2] = c2 * t21 - s2 * t22;
                G[q1][q2] = s2 * t21 + c2 * t22;
              } else {
                const int item = it - NP * NP, i = item / NP, m = item - i * NP;
                const int a = rr_player(m, r2, B2), b = rr_player(B2 - 1 - m, r2, B2);
                const int pp = a < b ? a : b, qq = a < b ? b : a;
                const double c = cs[m][0], sn = cs[m][1];
                const double vp = V[i][pp], vq = V[i][qq];
                V[i][pp] = c * vp - sn * vq;
                V[i][qq] = sn * vp + c * vq;
              }
            }
            __syncthreads();
        }
        const int rot = s_rot;
        if (tid == 0 && rot) {
            s_any = 1;
            if (sweep == 0 && slice == 0) rotated[0] = 1;
        }
        __syncthreads();
        if (!rot) break;
    }
    if (!s_any) return;
    if (tid == 0) {
        lr[P] = gidx;
        lr[Qb] = gidx;
    }

    // 3. vectors and rows of Q times V: thread (wave w, lane) makes entries
    //    x0 + lane + 64 v of the new vectors JW w .. JW w + JW - 1
    const int lane = tid & 63, j0 = (tid >> 6) * JW;
    for (int pass = 0; pass < 2; ++pass) {
        double* base = pass == 0 ? W : Qm;
        const int Lx = pass == 0 ? L : k;
        int ua, ub;
        span(Lx, ua, ub);
        for (int x0 = ua; x0 < ub; x0 += XC) {
            stage(base, Lx, x0, ub);
            __syncthreads();
            // all NV entries of the thread at once, so that each row of V
            // is read once per chunk (a copy of V in registers would take
            // 2b x JW doubles)
            constexpr int NV = XC / 64;
            double y[NV][JW];
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int u = 0; u < JW; ++u) y[v][u] = 0.0;
#pragma unroll 2
            for (int i = 0; i < B2; ++i) {
                double vr[JW];
#pragma unroll
                for (int u = 0; u < JW; ++u) vr[u] = V[i][j0 + u];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const double t = T[i][lane + 64 * v];
#pragma unroll
                    for (int u = 0; u < JW; ++u) y[v][u] = fma(t, vr[u], y[v][u]);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int x = x0 + lane + 64 * v;
#pragma unroll
                for (int u = 0; u < JW; ++u) {
                    const int c = col(j0 + u);
                    if (c < k && x < ub) base[static_cast<int64_t>(c) * Lx + x] = y[v][u];
                }
            }
            __syncthreads();
        }
    }
}

// norms, descending order (bitonic sort in LDS) and the outputs; one
// workgroup per sector
__global__ __launch_bounds__(512) void k_svd_finish(const SvdProb* __restrict__ probs, const double* __restrict__ Wg,
                                                     const double* __restrict__ Qg, double* __restrict__ Ug,
                                                     double* __restrict__ Sg, double* __restrict__ Vtg,
                                                     const double* __restrict__ shift) {
    constexpr int NT = 512, NW = NT / 64;
    __shared__ double sval[kSvdMaxK];
    __shared__ int order[kSvdMaxK];
    const SvdProb p = probs[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int k = p.k, L = p.L;
    const double* W = Wg + p.w_off;
    const double* Q = Qg + p.q_off;
    int kq = 1;
    while (kq < k) kq <<= 1;
    for (int j = wave; j < kq; j += NW) {
        double n2 = 0.0;
        if (j < k)
            for (int x = lane; x < L; x += 64) n2 = fma(W[static_cast<int64_t>(j) * L + x], W[static_cast<int64_t>(j) * L + x], n2);
        n2 = wave_sum(n2);
        if (lane == 0) {
            sval[j] = j < k ? sqrt(n2) : -1.0;
            order[j] = j;
        }
    }
    __syncthreads();
    for (int size = 2; size <= kq; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < kq; i += NT) {
                const int jx = i ^ stride;
                if (jx > i) {
                    const bool desc = (i & size) == 0;
                    const double vi = sval[i], vj = sval[jx];
                    if (desc ? (vi < vj) : (vi > vj)) {
                        sval[i] = vj;
                        sval[jx] = vi;
                        const int t = order[i];
                        order[i] = order[jx];
                        order[jx] = t;
                    }
                }
            }
            __syncthreads();
        }
    const double c = shift ? shift[blockIdx.x] : 0.0;
    for (int j = tid; j < k; j += NT) Sg[p.s_off + j] = sval[j] - c;
    // normalised vectors on one side, rotation rows on the other (in eigen
    // mode the vectors are rows and only the rotation side, U, is wanted)
    for (int64_t idx = tid; Vtg != nullptr && idx < static_cast<int64_t>(k) * L; idx += NT) {
        const int j = static_cast<int>(idx / L), x = static_cast<int>(idx - static_cast<int64_t>(j) * L);
        const double sv = sval[j];
        const double val = sv > 0.0 ? W[static_cast<int64_t>(order[j]) * L + x] / sv : 0.0;
        if (p.rows_are_vectors) Vtg[p.vt_off + static_cast<int64_t>(j) * p.N + x] = val;   // Vt[j][x], x < N
        else Ug[p.u_off + static_cast<int64_t>(x) * k + j] = val;                          // U[x][j], x < M
    }
    for (int64_t idx = tid; idx < static_cast<int64_t>(k) * k; idx += NT) {
        const int j = static_cast<int>(idx / k), i = static_cast<int>(idx - static_cast<int64_t>(j) * k);
        const double g = Q[static_cast<int64_t>(order[j]) * k + i];
        if (p.rows_are_vectors) Ug[p.u_off + static_cast<int64_t>(i) * k + j] = g;   // U[i][j] = G[v][i], i < M = k
        else Vtg[p.vt_off + static_cast<int64_t>(j) * p.N + i] = g;                   // Vt[j][i] = G[v][i], i < N = k
    }
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_svd(int src_dtype, const void* src, const SvdProb* probs, const int32_t* pair_start,
                      int32_t n_probs, int32_t n_pairs, int32_t max_kp, double* W, double* Q, double* U, double* S,
                      double* Vt, double* scale, double* shift, double* Gpart, int32_t* lastrot, int32_t* flag,
                      int32_t* flag_host, int32_t max_sweeps, int32_t* sweeps_done, hipStream_t s) {
    if (n_probs <= 0) return hipSuccess;
    dim3 lgrid(256, static_cast<unsigned>(n_probs));
    hipLaunchKernelGGL(k_fill_i32, dim3(static_cast<unsigned>((2 * n_probs + 63) / 64)), dim3(64), 0, s,
                       reinterpret_cast<int32_t*>(scale), 2 * n_probs, 0);
    if (src_dtype == 0)
        hipLaunchKernelGGL((k_svd_load<float>), lgrid, dim3(256), 0, s, static_cast<const float*>(src), probs, W, Q,
                           scale);
    else
        hipLaunchKernelGGL((k_svd_load<uint16_t>), lgrid, dim3(256), 0, s, static_cast<const uint16_t*>(src), probs, W,
                           Q, scale);
    hipLaunchKernelGGL(k_fill_i32, dim3(static_cast<unsigned>((2 * n_pairs + 255) / 256)), dim3(256), 0, s, lastrot,
                       2 * n_pairs, -1);
    if (shift)
        hipLaunchKernelGGL(k_eig_shift, dim3(static_cast<unsigned>(n_probs)), dim3(256), 0, s, probs, W, scale, shift);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int sweep = 0;
    // pair_start counts block pairs; max_kp is the largest (even) block count
    const dim3 rgrid(static_cast<unsigned>(n_pairs), kSvdSlices);
    while (sweep < max_sweeps && max_kp > 1 && n_pairs > 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, flag, 1, 0);
        for (int r = 0; r < max_kp - 1; ++r) {
            const int gidx = sweep * (max_kp - 1) + r;
            hipLaunchKernelGGL(k_svd_bround<0>, rgrid, dim3(256), 0, s, probs, n_probs, pair_start, r, W, Q, scale, Gpart,
                               flag, lastrot, gidx, max_kp - 1);
            hipLaunchKernelGGL(k_svd_bround<1>, rgrid, dim3(256), 0, s, probs, n_probs, pair_start, r, W, Q, scale, Gpart,
                               flag, lastrot, gidx, max_kp - 1);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ++sweep;
        // the sweep count is decided on the host: one small copy per sweep
        e = hipMemcpyAsync(flag_host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (*flag_host == 0) break;
    }
    if (sweeps_done) *sweeps_done = sweep;
    hipLaunchKernelGGL(k_svd_finish, dim3(static_cast<unsigned>(n_probs)), dim3(512), 0, s, probs, W, Q, U, S, Vt,
                       static_cast<const double*>(shift));
    return hipGetLastError();
}

// Polar decomposition from the block SVD (T = U diag(S) Vt): the isometric
// factor W = U Vt and the positive factor P = V diag(S) Vt (T = W P, rows >=
// columns) or U diag(S) U^T (T = P W), as FP64 products over 64 x 64 output
// tiles, 16-deep slices of the inner dimension staged in LDS, 4 x 4 outputs
// per thread.
__global__ __launch_bounds__(256) void k_polar_gemm(const PolarGemm* __restrict__ probs,
                                                    const PolarTile* __restrict__ tiles,
                                                    const double* __restrict__ uv, const double* __restrict__ S,
                                                    double* __restrict__ W, double* __restrict__ P) {
    constexpr int TT = kPolarTile, TK = 16;
    __shared__ double As[TK][TT + 1];
    __shared__ double Bs[TK][TT + 1];
    const PolarTile t = tiles[blockIdx.x];
    const PolarGemm p = probs[t.prob];
    const int tid = static_cast<int>(threadIdx.x), tx = tid & 15, ty = tid >> 4;
    double acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    for (int l0 = 0; l0 < p.kk; l0 += TK) {
        for (int e = tid; e < TT * TK; e += 256) {
            const int i = e % TT, l = e / TT, gi = t.i0 + i, gl = l0 + l;
            double v = 0.0;
            if (gi < p.m && gl < p.kk) {
                v = uv[p.a_off + static_cast<int64_t>(gi) * p.as0 + static_cast<int64_t>(gl) * p.as1];
                if (p.d_off >= 0) v *= S[p.d_off + gl];
            }
            As[l][i] = v;
        }
        for (int e = tid; e < TT * TK; e += 256) {
            const int j = e % TT, l = e / TT, gj = t.j0 + j, gl = l0 + l;
            Bs[l][j] = (gj < p.n && gl < p.kk)
                           ? uv[p.b_off + static_cast<int64_t>(gl) * p.bs0 + static_cast<int64_t>(gj) * p.bs1]
                           : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int l = 0; l < TK; ++l) {
            double a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[l][ty + 16 * r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[l][tx + 16 * c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
    double* C = p.which == 0 ? W : P;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gi = t.i0 + ty + 16 * r, gj = t.j0 + tx + 16 * c;
            if (gi < p.m && gj < p.n) C[p.c_off + static_cast<int64_t>(gi) * p.ldc + gj] = acc[r][c];
        }
}

hipError_t launch_polar(const PolarGemm* probs, const PolarTile* tiles, int32_t n_tiles, const double* uv,
                        const double* S, double* W, double* P, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_polar_gemm, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s, probs, tiles, uv, S, W, P);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// K9: SU(2) PERMUTE with recoupling.  For one label tuple, the n input
// blocks P^e are combined with the FP64 coefficients Gamma[f][e] of the
// permutation and tree change into the n output blocks.  The output's axis k
// is the input's axis perm[k]; the host hands over the input strides already
// in output-axis order, so the kernel only walks the output block row-major.
// Threads run along the output's innermost axis; a workgroup takes up to
// kRecoupleChunk elements of one tuple, several per thread, so that the
// tuple's metadata is read once for many elements.
// ---------------------------------------------------------------------------
// U output positions per thread per pass (256 apart, so lanes stay on
// consecutive positions); all their n loads are issued before any use.  A
// position is decoded once (mixed radix over the output's dims) into its
// offset inside the first input and the first output block; blocks that
// share strides reuse it.
// RK: the block rank when it is exactly 4 (the decode and the address sums
// then run over 4 dims with no rank test, which is what the element rate of
// the rank-4 trees needs: the general form measured 1.55 against 1.0 ms on
// config 5's recoupling), or kMaxRecoupleRank for any rank up to it.
template <int NB, int RK, typename Ti, typename To>
__device__ __forceinline__ void recouple_elems(const FmGroup& g, const FmBlk* __restrict__ ib,
                                               const FmBlk* __restrict__ ob, const double* __restrict__ cf,
                                               const Ti* __restrict__ src, To* __restrict__ dst, int start,
                                               int end) {
    constexpr int U = NB <= 2 ? 8 : NB <= 4 ? 4 : NB <= 8 ? 2 : 1;
    constexpr int R = RK;
    const int n = g.n, rank = RK == 4 ? 4 : g.rank;
    // offsets of position e in block b, for all blocks sharing b's strides or not
    auto decode = [&](int e, int (&t)[R]) {
        int r = e;
#pragma unroll
        for (int k = R - 1; k >= 1; --k) {
            if (k < rank) {
                const int q = div_by(r, g.mag[k], g.shf[k]);
                t[k] = r - q * g.d[k];
                r = q;
            } else {
                t[k] = 0;
            }
        }
        t[0] = r;
    };
    auto rel = [&](const FmBlk& b, const int (&t)[R]) {
        uint32_t o = 0;
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (k < rank) o += static_cast<uint32_t>(t[k] * b.stride[k]);
        return o;
    };
    for (int e0 = start + static_cast<int>(threadIdx.x); e0 < end; e0 += 256 * U) {
        float xs[U][NB];
        int pos[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + 256 * u;
            pos[u] = e < end ? e : -1;
            int t[R];
            decode(e < end ? e : start, t);
            const uint32_t ri0 = rel(ib[0], t);
#pragma unroll
            for (int i = 0; i < NB; ++i)
                xs[u][i] = i < n ? Conv<Ti, float>::f(src[ib[i].off + (g.same_in ? ri0 : rel(ib[i], t))]) : 0.f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (pos[u] < 0) continue;
            int t[R];
            decode(pos[u], t);
            const uint32_t ro0 = rel(ob[0], t);
#pragma unroll
            for (int f = 0; f < NB; ++f) {
                if (f >= n) break;
                double y = 0.0;
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    if (i < n) y = fma(cf[f * n + i], static_cast<double>(xs[u][i]), y);
                // streaming store: the output is not read again by this kernel
                __builtin_nontemporal_store(Conv<float, To>::f(static_cast<float>(y)),
                                            &dst[ob[f].off + (g.same_out ? ro0 : rel(ob[f], t))]);
            }
        }
    }
}

// NBMAX: the largest n (blocks per label tuple) the instance takes.  The
// plan launches tuples of at most kRecoupleSmallN blocks (93 % of config 5's
// output elements) through an instance held to 64 VGPRs, eight waves per
// SIMD: the kernel is bound by memory latency, and its small-n paths need
// few registers, while one kernel for every n takes the register count of
// its n = 32 path (112 VGPRs, four waves per SIMD).  The larger tuples go
// through the general instance.
template <int NBMAX, typename Ti, typename To>
__global__ __launch_bounds__(256, NBMAX <= kRecoupleSmallN ? 8 : 1) void k_recouple(
    const FmGroup* __restrict__ groups, const FmBlk* __restrict__ in_blks, const FmBlk* __restrict__ out_blks,
    const double* __restrict__ coef, const FmTask* __restrict__ tasks, PtrTable bufs, int in_buf, int out_buf) {
    __shared__ double cf[NBMAX * NBMAX];
    const FmTask t = tasks[blockIdx.x];
    const FmGroup& g = groups[t.group];
    for (int k = threadIdx.x; k < g.n * g.n; k += 256) cf[k] = coef[g.coef_first + k];
    __syncthreads();
    const Ti* __restrict__ src = static_cast<const Ti*>(bufs.p[in_buf]);
    To* __restrict__ dst = static_cast<To*>(const_cast<void*>(bufs.p[out_buf]));
    const FmBlk* __restrict__ ib = in_blks + g.in_first;
    const FmBlk* __restrict__ ob = out_blks + g.out_first;
    const int end = t.start + t.count;
    const int n = g.n;
    if (g.rank == 4) {
        if (n <= 1) recouple_elems<1, 4, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
        else if (n <= 2) recouple_elems<2, 4, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
        else if (n <= 4) recouple_elems<4, 4, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
        else if (n <= 8) recouple_elems<8, 4, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
        else if (n <= 16) recouple_elems<16, 4, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
        else if constexpr (NBMAX > 16) recouple_elems<kMaxRecouple, 4, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
        return;
    }
    constexpr int RG = kMaxRecoupleRank;
    if (n <= 1) recouple_elems<1, RG, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
    else if (n <= 2) recouple_elems<2, RG, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
    else if (n <= 4) recouple_elems<4, RG, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
    else if (n <= 8) recouple_elems<8, RG, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
    else if (n <= 16) recouple_elems<16, RG, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
    else if constexpr (NBMAX > 16) recouple_elems<kMaxRecouple, RG, Ti, To>(g, ib, ob, cf, src, dst, t.start, end);
}

// LDS-tiled K9 (see FtGroup): a workgroup moves one box of all n input
// blocks of a label tuple into LDS, issuing every load of the box before it
// stores any of them (16 per thread in flight), in the order that makes
// consecutive lanes read consecutive input addresses; it then combines the
// n values of each box position with the FP64 coefficients (staged in LDS)
// and writes the n output blocks in output order.  Per-block offsets and
// strides are decoded once per task into LDS.  The combination is unrolled
// for n up to NB (the smallest power of two >= n).
template <int NB, typename To>
__device__ __forceinline__ void recouple_combine(const float* __restrict__ tile, const double* __restrict__ cf,
                                                 const int64_t* __restrict__ obase, const int32_t (*ostr)[3],
                                                 To* __restrict__ dst, int n, int E, int T2, int T3, int v1, int v2,
                                                 int v3, uint32_t m0, int s0, uint32_t m1, int s1) {
    for (int q = threadIdx.x; q < E; q += 256) {
        const int r = div_by(q, m0, s0);
        const int l3 = q - r * T3;
        const int l1 = div_by(r, m1, s1);
        const int l2 = r - l1 * T2;
        if (l1 >= v1 || l2 >= v2 || l3 >= v3) continue;
        double x[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = i < n ? static_cast<double>(tile[i * E + q]) : 0.0;
#pragma unroll
        for (int f = 0; f < NB; ++f) {
            if (f >= n) break;
            double y = 0.0;
#pragma unroll
            for (int i = 0; i < NB; ++i)
                if (i < n) y = fma(cf[f * n + i], x[i], y);
            dst[obase[f] + (l1 * ostr[f][0] + l2 * ostr[f][1] + l3 * ostr[f][2])] = Conv<float, To>::f(static_cast<float>(y));
        }
    }
}

// NBMAX: the largest n the instance takes; tuples of at most
// kRecoupleTiledSmallN blocks run in an instance held to eight waves per
// SIMD (like the element-wise kernel, this one waits on memory latency)
template <int NBMAX, typename Ti, typename To>
__global__ __launch_bounds__(256, NBMAX <= kRecoupleTiledSmallN ? 8 : 1) void k_recouple_tiled(
    const FtGroup* __restrict__ groups, const FmBlk* __restrict__ in_blks, const FmBlk* __restrict__ out_blks,
    const double* __restrict__ coef, const FtTask* __restrict__ tasks, PtrTable bufs, int in_buf, int out_buf) {
    constexpr int U = 16;
    __shared__ float tile[kFtElems];
    __shared__ double cf[NBMAX * NBMAX];
    __shared__ int64_t ibase[NBMAX], obase[NBMAX];
    __shared__ int32_t istr[NBMAX][3], ostr[NBMAX][3];
    const FtTask t = tasks[blockIdx.x];
    const FtGroup& g = groups[t.group];
    const int n = g.n;
    const int a0 = g.ax[0], a1 = g.ax[1], a2 = g.ax[2], a3 = g.ax[3];
    const int T1 = g.t[1], T2 = g.t[2], T3 = g.t[3], E = g.esz;
    const int tid = threadIdx.x;
    for (int k = tid; k < n * n; k += 256) cf[k] = coef[g.coef_first + k];
    if (tid < 2 * n) {
        const bool in = tid < n;
        const int i = in ? tid : tid - n;
        // read through a pointer: indexing a copy of the record by the
        // axis numbers would put it in scratch memory
        const FmBlk* b = in ? in_blks + g.in_first + i : out_blks + g.out_first + i;
        const int64_t base = b->off + static_cast<int64_t>(t.o[0]) * b->stride[a0] +
                             static_cast<int64_t>(t.o[1]) * b->stride[a1] +
                             static_cast<int64_t>(t.o[2]) * b->stride[a2] + static_cast<int64_t>(t.o[3]) * b->stride[a3];
        (in ? ibase : obase)[i] = base;
        int32_t* st = in ? istr[i] : ostr[i];
        st[0] = b->stride[a1];
        st[1] = b->stride[a2];
        st[2] = b->stride[a3];
    }
    __syncthreads();
    // extents of the box inside the blocks (edge tiles are clipped)
    const int v1 = min(T1, g.dim[a1] - t.o[1]), v2 = min(T2, g.dim[a2] - t.o[2]), v3 = min(T3, g.dim[a3] - t.o[3]);
    const Ti* __restrict__ src = static_cast<const Ti*>(bufs.p[in_buf]);
    To* __restrict__ dst = static_cast<To*>(const_cast<void*>(bufs.p[out_buf]));
    const int lf = g.ld[0], lm = g.ld[1];
    const int tf = g.t[lf], tm = g.t[lm];
    const int total = n * E;
    for (int b0 = 0; b0 < total; b0 += 256 * U) {
        float v[U];
        int pos[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = b0 + u * 256 + tid;
            pos[u] = -1;
            v[u] = 0.f;
            if (idx < total) {
                const int i = div_by(idx, g.mag[4], g.shf[4]);
                const int q = idx - i * E;
                const int r = div_by(q, g.mag[2], g.shf[2]);
                const int uf = q - r * tf;
                const int us = div_by(r, g.mag[3], g.shf[3]);
                const int um = r - us * tm;
                // box coordinates (slots 1..3) from the load-order ones
                const int l1 = lf == 1 ? uf : (lm == 1 ? um : us);
                const int l2 = lf == 2 ? uf : (lm == 2 ? um : us);
                const int l3 = lf == 3 ? uf : (lm == 3 ? um : us);
                if (l1 < v1 && l2 < v2 && l3 < v3) {
                    const int rel = l1 * istr[i][0] + l2 * istr[i][1] + l3 * istr[i][2];
                    v[u] = Conv<Ti, float>::f(src[ibase[i] + rel]);
                    pos[u] = i * E + (l1 * T2 + l2) * T3 + l3;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (pos[u] >= 0) tile[pos[u]] = v[u];
    }
    __syncthreads();
    const uint32_t m0 = g.mag[0], m1 = g.mag[1];
    const int s0 = g.shf[0], s1 = g.shf[1];
    if (n <= 1)
        recouple_combine<1, To>(tile, cf, obase, ostr, dst, n, E, T2, T3, v1, v2, v3, m0, s0, m1, s1);
    else if (n <= 2)
        recouple_combine<2, To>(tile, cf, obase, ostr, dst, n, E, T2, T3, v1, v2, v3, m0, s0, m1, s1);
    else if (n <= 4)
        recouple_combine<4, To>(tile, cf, obase, ostr, dst, n, E, T2, T3, v1, v2, v3, m0, s0, m1, s1);
    else if constexpr (NBMAX > 4) {
        if (n <= 8)
            recouple_combine<8, To>(tile, cf, obase, ostr, dst, n, E, T2, T3, v1, v2, v3, m0, s0, m1, s1);
        else
            recouple_combine<kMaxRecoupleTiled, To>(tile, cf, obase, ostr, dst, n, E, T2, T3, v1, v2, v3, m0, s0, m1,
                                                s1);
    }
}

template <typename Ti, typename To>
hipError_t launch_rct(const FtGroup* groups, const FmBlk* in_blks, const FmBlk* out_blks, const double* coef,
                      const FtTask* tasks, int32_t n_small, int32_t n_tasks, const PtrTable& bufs, int32_t in_buf,
                      int32_t out_buf, hipStream_t s) {
    if (n_small > 0) {
        hipLaunchKernelGGL((k_recouple_tiled<kRecoupleTiledSmallN, Ti, To>), dim3(static_cast<unsigned>(n_small)),
                           dim3(256), 0, s, groups, in_blks, out_blks, coef, tasks, bufs, in_buf, out_buf);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_tasks > n_small)
        hipLaunchKernelGGL((k_recouple_tiled<kMaxRecoupleTiled, Ti, To>), dim3(static_cast<unsigned>(n_tasks - n_small)),
                           dim3(256), 0, s, groups, in_blks, out_blks, coef, tasks + n_small, bufs, in_buf, out_buf);
    return hipGetLastError();
}

template <typename Ti, typename To>
hipError_t launch_rce(const FmGroup* groups, const FmBlk* in_blks, const FmBlk* out_blks, const double* coef,
                      const FmTask* tasks, int32_t n_small, int32_t n_tasks, const PtrTable& bufs, int32_t in_buf,
                      int32_t out_buf, hipStream_t s) {
    if (n_small > 0) {
        hipLaunchKernelGGL((k_recouple<kRecoupleSmallN, Ti, To>), dim3(static_cast<unsigned>(n_small)), dim3(256), 0, s,
                           groups, in_blks, out_blks, coef, tasks, bufs, in_buf, out_buf);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_tasks > n_small)
        hipLaunchKernelGGL((k_recouple<kMaxRecouple, Ti, To>), dim3(static_cast<unsigned>(n_tasks - n_small)), dim3(256),
                           0, s, groups, in_blks, out_blks, coef, tasks + n_small, bufs, in_buf, out_buf);
    return hipGetLastError();
}

bool recouple_dtypes_supported(int src_dtype, int dst_dtype) {
    return (src_dtype == 0 && (dst_dtype == 0 || dst_dtype == 1)) || (src_dtype == 1 && dst_dtype == 1);
}

hipError_t launch_recouple_tiled(int src_dtype, int dst_dtype, const FtGroup* groups, const FmBlk* in_blks,
                                 const FmBlk* out_blks, const double* coef, const FtTask* tasks, int32_t n_small,
                                 int32_t n_tasks, const PtrTable& bufs, int32_t in_buf, int32_t out_buf,
                                 hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    if (src_dtype == 0 && dst_dtype == 0)
        return launch_rct<float, float>(groups, in_blks, out_blks, coef, tasks, n_small, n_tasks, bufs, in_buf, out_buf, s);
    if (src_dtype == 0 && dst_dtype == 1)
        return launch_rct<float, uint16_t>(groups, in_blks, out_blks, coef, tasks, n_small, n_tasks, bufs, in_buf, out_buf,
                                           s);
    if (src_dtype == 1 && dst_dtype == 1)
        return launch_rct<uint16_t, uint16_t>(groups, in_blks, out_blks, coef, tasks, n_small, n_tasks, bufs, in_buf,
                                              out_buf, s);
    return hipErrorInvalidValue;
}

hipError_t launch_recouple(int src_dtype, int dst_dtype, const FmGroup* groups, const FmBlk* in_blks,
                           const FmBlk* out_blks, const double* coef, const FmTask* tasks, int32_t n_small,
                           int32_t n_tasks, const PtrTable& bufs, int32_t in_buf, int32_t out_buf, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    if (src_dtype == 0 && dst_dtype == 0)
        return launch_rce<float, float>(groups, in_blks, out_blks, coef, tasks, n_small, n_tasks, bufs, in_buf, out_buf, s);
    if (src_dtype == 0 && dst_dtype == 1)
        return launch_rce<float, uint16_t>(groups, in_blks, out_blks, coef, tasks, n_small, n_tasks, bufs, in_buf, out_buf,
                                           s);
    if (src_dtype == 1 && dst_dtype == 1)
        return launch_rce<uint16_t, uint16_t>(groups, in_blks, out_blks, coef, tasks, n_small, n_tasks, bufs, in_buf,
                                              out_buf, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Fixed device memory of the entry point that allocates nothing.  The array
// is a module variable: every GPU the library runs on holds its own copy for
// the life of the process.  On the host its name is only a stand-in for the
// symbol; the device address comes from hipGetSymbolAddress, looked up once
// per device with that device current, and only that address is ever handed
// to kernels or copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch(void** ptr) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

// Zero fill by a kernel (also inside captured graphs, where a memset node is
// avoided); n16 16-byte words from a 16-byte aligned address.
__global__ __launch_bounds__(256) void k_zero16(u32x4* __restrict__ p, int64_t n16) {
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n16;
         i += static_cast<int64_t>(gridDim.x) * 256)
        p[i] = z;
}

// Small contractions: one workgroup per task, a thread per output entry
// (two passes of 256), FP32 fused multiply-adds in a fixed order (pairs in
// plan order, k ascending).  The pair records are uniform across the
// workgroup, so their fields load into scalar registers; the k loop is
// unrolled 16 times so that 16 A and 16 B loads are in flight at once.
// Measured on a contraction of 85 blocks of 16 x 16 (2.66 MFLOP): 7.6 us per
// call back to back, against 8.1 us unrolled 4 times, 8.0 us with the next
// pair's record requested ahead, 12.8 us walking all (pair, k) terms as one
// sequence from LDS, 10.8 us staging the operand blocks in LDS first; a
// trivial torch kernel takes 6.4 us the same way.
__global__ __launch_bounds__(256) void k_contract_small(const SmallTask* __restrict__ tasks,
                                                        const SmallPair* __restrict__ pairs, PtrTable bufs) {
    const SmallTask t = tasks[blockIdx.x];
    float* C = static_cast<float*>(const_cast<void*>(bufs.p[t.c_buf])) + t.c_off;
    for (int e = t.e0 + static_cast<int>(threadIdx.x); e < t.e1; e += 256) {
        const int m = e / t.N, n = e - m * t.N;
        float acc = 0.f;
        for (int q = 0; q < t.pair_count; ++q) {
            const SmallPair p = pairs[t.pair_first + q];
            const float* A = static_cast<const float*>(bufs.p[p.a_buf]) + p.a_off + static_cast<int64_t>(m) * p.a_rs;
            const float* B = static_cast<const float*>(bufs.p[p.b_buf]) + p.b_off + static_cast<int64_t>(n) * p.b_cs;
#pragma unroll 16
            for (int k = 0; k < p.K; ++k)
                acc = __builtin_fmaf(A[static_cast<int64_t>(k) * p.a_cs], B[static_cast<int64_t>(k) * p.b_rs], acc);
        }
        C[static_cast<int64_t>(m) * t.c_rs + static_cast<int64_t>(n) * t.c_cs] = acc;
    }
}

hipError_t launch_contract_small(const SmallTask* tasks, int32_t n_tasks, const SmallPair* pairs,
                                 const PtrTable& bufs, hipStream_t s) {
    if (n_tasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_contract_small, dim3(static_cast<unsigned>(n_tasks)), dim3(256), 0, s, tasks, pairs, bufs);
    return hipGetLastError();
}

hipError_t launch_zero16(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if ((bytes & 15u) != 0 || (reinterpret_cast<uintptr_t>(p) & 15u) != 0) return hipErrorInvalidValue;
    const int64_t n16 = static_cast<int64_t>(bytes / 16);
    const int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero16, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, static_cast<u32x4*>(p), n16);
    return hipGetLastError();
}

}  // namespace sym
