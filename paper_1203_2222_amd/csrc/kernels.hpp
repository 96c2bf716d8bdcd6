// Device work descriptors shared by the host planner and the HIP kernels.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace sym {

constexpr int kMaxBufs = 256;       // distinct base pointers one launch may address
constexpr int kMaxCopyDims = 6;     // dims of a coalesced block copy
constexpr int kMaxRecouple = 32;    // blocks of one label tuple on either side of a recoupling
constexpr int kMaxRecoupleTiled = 16;   // the same for the LDS-tiled kernel (its LDS tables scale with it)
constexpr int kMaxRecoupleRank = 8;
constexpr int kRecoupleChunk = 16384;  // elements of one label tuple per workgroup task
constexpr int kRecoupleSmallN = 16;   // label tuples of at most this many blocks take the high-occupancy kernel

// Base pointers of one launch, passed by value as a kernel argument.
struct PtrTable {
    const void* p[kMaxBufs];
};

// One block copy dst = convert(src) over a strided box (dim kMaxCopyDims-1 innermost).
struct CopyOp {
    int64_t src_off, dst_off;
    int64_t sstride[kMaxCopyDims];
    int64_t dstride[kMaxCopyDims];
    int32_t size[kMaxCopyDims];
    // floor(n / size[d]) = (n * mag[d]) >> (31 + shf[d]) for 0 <= n < 2^31
    uint32_t mag[kMaxCopyDims];
    int32_t shf[kMaxCopyDims];
    int32_t src_buf, dst_buf;
    int32_t count;
    int32_t ndim;
    int32_t tj;          // tiled copies: the dim that is contiguous in the source
    int32_t rowcopy;     // rows of a contiguous source run along the destination's rows
    int64_t src_len;     // elements readable from the source buffer's base pointer
    int32_t neg;         // 1: the block changes sign (fermionic swap factors)
    // vectorized transposes of small blocks: the dim that continues the
    // destination-contiguous dim (dstride == size of the innermost dim) and
    // the one that continues the source-contiguous dim tj (sstride ==
    // size[tj]), merged into them so that a tile spans both; -1 for none
    int32_t ihi, jhi;
    int32_t pad;
};

// A slice [start, start+count) of one CopyOp's elements (in destination order).
struct CopyTask {
    int32_t op, start, count, pad;
};

// Row copies: rows [row0, row0 + nrows), columns [col0, col0 + ncols) of a
// CopyOp whose inner dim is contiguous on both sides and whose source rows
// follow each other (nrows > 1 only with whole rows).
struct RowTask {
    int32_t op, row0, nrows, col0, ncols, pad0, pad1, pad2;
};
constexpr int kRowStage = 8192;   // source elements one row task stages through LDS

// One 64 x 64 tile of a transposing copy: rows along the destination's
// contiguous dim (index kMaxCopyDims-1), columns along the source's (tj).
struct TileTask {
    int32_t op, outer, jt, it;
};
constexpr int kTile = 64;
// rows (destination-contiguous extent) of a vectorized transposing tile, by
// source element size.  Longer destination segments write fewer partial
// cache lines: for BF16 sources 256 rows measured 7 % faster than 128 and
// 64 rows 23 % slower (batched B operand, 21.4 GB); 512 was slower again.
constexpr int vtile_rows(int src_elem_bytes) { return src_elem_bytes == 2 ? 256 : 64; }
// columns (source-contiguous extent) of a vectorized transposing tile: 128
// BF16 columns (256-byte source segments) measured 2 to 3 % slower on the
// batched fuse, with 256 rows (one workgroup per CU) or with 128
constexpr int vtile_cols(int) { return 64; }

// One sector GEMM: C[m][n] = sum_k A[m][k] * B[n][k] (both operands K-contiguous).
// With `indirect` set, element (m, n) is stored at
//   c_off + row.r0 + row.r1 * col.c1 + row.r2 * col.c2 + col.c0
// (row = rows[ri_off + m], col = cols[ci_off + n]): the split into a
// canonical block list, done by the epilogue instead of a separate pass.
struct GemmProb {
    int64_t a_off, b_off, c_off;
    int64_t ri_off, ci_off;
    int32_t M, N, K;
    int32_t lda, ldb, ldc;
    int32_t a_buf, b_buf, c_buf;
    int32_t indirect;
};

// Canonical block list of a row-legs-first tensor: block (rt, ct) of a sector
// starts at base(rt) + d(rt) * colcum(ct) and is row-major, so the element at
// row offset t_r in rt and column offset t_c in ct sits at
// base(rt) + t_r * d(ct) + d(rt) * colcum(ct) + t_c.  All terms are 32-bit:
// the planner uses this form only for outputs below 2^29 elements whose
// tuple dimensions and column offsets are below 2^24 (24-bit multiplies).
struct EpiRow {
    int32_t r0;   // base(rt)
    int32_t r1;   // t_r
    int32_t r2;   // d(rt)
    int32_t pad;
};
struct EpiCol {
    int32_t c2;   // colcum(ct)
    int32_t c0;   // t_c
    int32_t c1;   // d(ct)
    int32_t pad;
};

struct GemmTile {
    int32_t prob, tm, tn, pad;
};

// SU(2) PERMUTE with recoupling of one label tuple: n input blocks (one per
// intermediate spin e of the input tree) and n output blocks (one per f of
// the output tree).
struct FmGroup {
    int32_t n;
    int32_t rank;        // block rank (dims past it are 1)
    int32_t d[kMaxRecoupleRank];      // block dims in output-axis order
    uint32_t mag[kMaxRecoupleRank];   // division by d[k] for k >= 1 (multiplier and shift,
    int32_t shf[kMaxRecoupleRank];    // floor(x / d) = (x * mag) >> (31 + shf) for x < 2^31)
    int32_t same_in;     // all input blocks share their strides
    int32_t same_out;    // all output blocks share their strides
    int32_t in_first;    // index of its first FmBlk among inputs
    int32_t out_first;   // index of its first FmBlk among outputs
    int32_t coef_first;  // n*n coefficients, row f, column e
};

// Element strides of a block along the output's axes 0..3 (for an input
// block: its stride along input axis perm[k]); every element of the block
// lies below 2^31 elements from its first one.
struct FmBlk {
    int64_t off;
    int32_t stride[kMaxRecoupleRank];
};

struct FmTask {
    int32_t group, start, count, pad;
};

// LDS-tiled recoupling: a task is a tile of one label tuple, the same box of
// every one of its n input and n output blocks.  The box fixes the index
// along output axis ax[0] and spans t[1] x t[2] x t[3] indices along output
// axes ax[1], ax[2], ax[3] (ascending, so ax[3] is the output's innermost
// axis).  Loads walk the box fastest along the tile axis of smallest input
// stride (ld[0], then ld[1], then ld[2]: slots 1..3), so that consecutive
// lanes read consecutive input addresses; the combination and the stores
// walk it in output order.
constexpr int kFtElems = 4096;   // floats of one tile over all n blocks (16 KB of LDS)
constexpr int kRecoupleTiledSmallN = 4;   // tuples of at most this many blocks take the high-occupancy tiled kernel
struct FtGroup {
    int32_t n;
    int32_t dim[4];      // output block dims, output-axis order
    int32_t ax[4];       // ax[0]: axis fixed per task; ax[1..3]: tile axes
    int32_t t[4];        // nominal tile extents along ax[1..3] (t[0] = 1)
    int32_t ld[3];       // load order: tile slots (1..3), fastest first
    int32_t esz;         // t[1] t[2] t[3]
    // floor(x / d) by multiplier and shift for d = t[3], t[2], t[ld[0]],
    // t[ld[1]] and esz (x < 2^31)
    uint32_t mag[5];
    int32_t shf[5];
    int32_t in_first, out_first, coef_first;
};
struct FtTask {
    int32_t group;
    int32_t o[4];        // index along ax[0]; tile origin along ax[1..3]
    int32_t pad[3];
};

// Small contractions in one launch (eq:tensormult block by block): a task is
// a range of entries of one output block, C(m, n) = sum over its block pairs
// of sum_k A(m, k) B(k, n), each operand block read as a strided matrix
// straight from the caller's tensors (no fused workspace, no split).
struct SmallTask {
    int64_t c_off;
    int32_t c_rs, c_cs;          // C(m, n) at c_off + m c_rs + n c_cs
    int32_t N;                   // columns of the block
    int32_t e0, e1;              // entries [e0, e1) of the block, row-major
    int32_t pair_first, pair_count;
    int32_t c_buf;
    int32_t pad[2];
};
struct SmallPair {
    int64_t a_off, b_off;
    int32_t a_rs, a_cs;          // A(m, k) at a_off + m a_rs + k a_cs
    int32_t b_rs, b_cs;          // B(k, n) at b_off + k b_rs + n b_cs
    int32_t K;
    int32_t a_buf, b_buf;
    int32_t pad;
};
constexpr int kSmallTaskElems = 512;   // entries of one task (two per thread)

// Launchers (kernels.hip).  Every launcher returns the hipError_t of the launch.
hipError_t launch_permute(int src_dtype, int dst_dtype, const CopyOp* ops, const CopyTask* tasks,
                          const int32_t* wg_begin, int32_t n_wg, const PtrTable& bufs, hipStream_t s);
hipError_t launch_copy_rows(int src_dtype, int dst_dtype, const CopyOp* ops, const RowTask* tasks, int32_t n_tasks,
                            int32_t grid, const PtrTable& bufs, hipStream_t s);
// merged: the tasks' ops have ihi or jhi set (all of them, or none)
hipError_t launch_transpose_vec(int src_dtype, int dst_dtype, bool merged, const CopyOp* ops, const TileTask* tasks,
                                int32_t n_tasks, int32_t grid, const PtrTable& bufs, hipStream_t s);
// grid: workgroups, each taking tasks w, w + grid, ...
hipError_t launch_permute_tiled(int src_dtype, int dst_dtype, const CopyOp* ops, const TileTask* tasks,
                                int32_t n_tasks, int32_t grid, const PtrTable& bufs, hipStream_t s);
hipError_t launch_gemm(int compute, int variant, const GemmProb* probs, const GemmTile* tiles,
                       int32_t n_tiles, int32_t grid, const EpiRow* rows, const EpiCol* cols,
                       const PtrTable& bufs, hipStream_t s);
// Recoupling element types (0 = F32, 1 = BF16; values are combined in FP64
// and rounded once to the output type): F32 -> F32, F32 -> BF16 and
// BF16 -> BF16.
bool recouple_dtypes_supported(int src_dtype, int dst_dtype);
// tasks[0, n_small) belong to tuples of at most kRecoupleTiledSmallN blocks
hipError_t launch_recouple_tiled(int src_dtype, int dst_dtype, const FtGroup* groups, const FmBlk* in_blks,
                                 const FmBlk* out_blks, const double* coef, const FtTask* tasks, int32_t n_small,
                                 int32_t n_tasks, const PtrTable& bufs, int32_t in_buf, int32_t out_buf,
                                 hipStream_t s);
hipError_t launch_contract_small(const SmallTask* tasks, int32_t n_tasks, const SmallPair* pairs,
                                 const PtrTable& bufs, hipStream_t s);
// tasks[0, n_small) belong to label tuples of at most kRecoupleSmallN blocks,
// tasks[n_small, n_tasks) to larger ones
hipError_t launch_recouple(int src_dtype, int dst_dtype, const FmGroup* groups, const FmBlk* in_blks,
                           const FmBlk* out_blks, const double* coef, const FmTask* tasks, int32_t n_small,
                           int32_t n_tasks, const PtrTable& bufs, int32_t in_buf, int32_t out_buf, hipStream_t s);

// Tile shape of a GEMM variant (rows x cols of C per workgroup).
struct GemmVariant {
    int mt, nt;
    const char* name;
};
int gemm_num_variants(int compute);
GemmVariant gemm_variant(int compute, int variant);
int gemm_default_variant(int compute);
// The kernel a variant launches, as its template instance (the name tools
// such as profilers print, without the namespace and parameter list).
const char* gemm_variant_kernel(int compute, int variant);
// Default for problems whose row lengths rule out the direct-load variants.
int gemm_default_variant_wide(int compute);
// Direct-load BF16 variants address each operand tile through a 32-bit
// buffer range: they take row lengths (lda, ldb) below gemm_direct_max_ld().
bool gemm_variant_direct(int compute, int variant);
int gemm_direct_max_ld();
// One sector of a block-wise SVD (one-sided Jacobi, FP64).  The k = min(M, N)
// vectors that get orthogonalised are the rows of the sector matrix when
// M <= N, its columns otherwise; each has length L = max(M, N).
struct SvdProb {
    int64_t src_off;              // element offset of the sector matrix (row-major, ld)
    int64_t w_off, q_off;         // FP64 workspace: vectors (k x L), rotations (k x k)
    int64_t u_off, s_off, vt_off; // outputs: U (M x k), S (k), Vt (k x N), row-major
    int32_t M, N, ld, k, L, rows_are_vectors;
    int32_t sym;                  // eigen mode: load (T + T^T) / 2 of a square sector, then shift it
    int32_t pad1;
};
constexpr int kSvdMaxK = 4096;    // k sorted in LDS
constexpr int kSvdBlock = 16;     // vectors per block of the block-Jacobi rounds
constexpr int kSvdSlices = 2;     // workgroups per pair of blocks (slices of the vector entries)
// Jacobi sweeps until one rotates nothing or max_sweeps; synchronises the
// stream once per sweep (the stopping decision is taken on the host).
// shift != NULL selects the eigen mode (every problem has sym set): each
// symmetric part S is factorised as S + c I, c its Frobenius norm (1 for a
// zero matrix, c per problem written to shift), S is returned as the
// singular values minus c and U holds the eigenvectors; Vt may be NULL.
hipError_t launch_svd(int src_dtype, const void* src, const SvdProb* probs, const int32_t* pair_start,
                      int32_t n_probs, int32_t n_pairs, int32_t max_kp, double* W, double* Q, double* U, double* S,
                      double* Vt, double* scale, double* shift, double* Gpart, int32_t* lastrot, int32_t* flag,
                      int32_t* flag_host, int32_t max_sweeps, int32_t* sweeps_done, hipStream_t s);
// Polar factors from a block SVD: per sector one or two FP64 products
// C = A diag(d) B with A(i, l) = a[a_off + i as0 + l as1] and
// B(l, j) = a[b_off + l bs0 + j bs1], both read from one buffer (U then Vt),
// d = S (or none when d_off < 0), C row-major with leading dimension ldc in
// out[which].
struct PolarGemm {
    int64_t a_off, b_off, c_off, d_off;
    int32_t m, n, kk, as0, as1, bs0, bs1, ldc, which, pad;
};
struct PolarTile {
    int32_t prob, i0, j0, pad;
};
constexpr int kPolarTile = 64;    // output tile edge of the polar products
hipError_t launch_polar(const PolarGemm* probs, const PolarTile* tiles, int32_t n_tiles, const double* uv,
                        const double* S, double* W, double* P, hipStream_t s);

// Resident workgroups per CU of a variant (persistent grid sizing).
int gemm_blocks_per_cu(int compute, int variant);

// Device memory of the entry point that allocates nothing: a fixed array of
// kNoAllocScratchBytes on every device, its address for the current device
// (looked up on the first call on that device).
constexpr size_t kNoAllocScratchBytes = size_t{64} << 20;
hipError_t noalloc_scratch(void** ptr);
// Zero `bytes` (a multiple of 16) from a 16-byte aligned device address.
hipError_t launch_zero16(void* p, size_t bytes, hipStream_t s);

}  // namespace sym
