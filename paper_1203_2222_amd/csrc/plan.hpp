// Host-side plans: everything a contraction or permute needs that depends
// only on the symmetry structure (block matching, offsets, tile lists,
// recoupling coefficients), built once, uploaded once and cached.  This is
// the thesis' "precompute once, reuse every iteration" (section "Permutation
// of indices" of the tree-decomposition chapter; Abelian chapter preface).
#pragma once

#include <functional>

#include "internal.hpp"
#include "kernels.hpp"

namespace sym {

// Device allocation owned by a plan, released through the context allocator.
struct DevMem {
    void* ptr = nullptr;
    size_t bytes = 0;
    std::function<void(void*)> release;
    DevMem() = default;
    DevMem(const DevMem&) = delete;
    DevMem& operator=(const DevMem&) = delete;
    ~DevMem() {
        if (ptr && release) release(ptr);
    }
};
using DevMemPtr = std::shared_ptr<DevMem>;
using Allocator = std::function<DevMemPtr(size_t)>;

// A host-to-device copy of a plan table.  Plans whose tables live in memory
// that other calls reuse (the entry point that allocates nothing) record
// their uploads instead of performing them, and repeat them before each
// launch; the host vectors they read belong to the plan and never change
// after it is built.
struct HostCopy {
    void* dst;
    const void* src;
    size_t bytes;
};
using Deferred = std::vector<HostCopy>;

// A batch of block copies launched together.
struct CopyProgram {
    std::vector<CopyOp> ops;
    std::vector<CopyTask> tasks;
    std::vector<int32_t> wg_begin;
    std::vector<TileTask> tile_tasks;
    std::vector<RowTask> row_tasks;
    std::vector<TileTask> vtile_tasks;   // transposes with unit-stride destination rows
    std::vector<TileTask> mtile_tasks;   // the same, for ops with merged row or column dims
    int32_t tile_grid = 0;   // workgroups of the tiled kernels (a multiple of 8 once there are 8 tasks)
    int32_t vtile_grid = 0, mtile_grid = 0;
    static constexpr int32_t kTileGridMax = 8192;
    int src_dtype = SYM_F32, dst_dtype = SYM_F32;
    // device copies
    DevMemPtr d_ops, d_tasks, d_wg, d_tile_tasks, d_row_tasks, d_vtile_tasks, d_mtile_tasks;

    // dst block j <- src block with labels dst.labels permuted back by perm
    void add(const Desc& src, const Desc& dst, const std::vector<int32_t>& perm, int src_buf, int dst_buf,
             int64_t src_base = 0, int64_t dst_base = 0);
    void finalize();
    void upload(const Allocator& alloc, Deferred* deferred = nullptr);
    bool empty() const { return ops.empty(); }
    // XCD-aware order of a tile list for a persistent grid; returns the grid
    static int32_t xcd_order(std::vector<TileTask>& list);
    hipError_t launch(const PtrTable& bufs, hipStream_t s) const;
};

struct GemmProgram {
    std::vector<GemmProb> probs;
    std::vector<GemmTile> tiles;
    int compute = SYM_F32;
    int variant = 0;
    int64_t flops = 0;
    std::vector<EpiRow> erows;
    std::vector<EpiCol> ecols;
    DevMemPtr d_probs, d_tiles, d_rows, d_cols;

    // One GEMM per sector of Z: Z = X * Y^T (X: M x K, Y: N x K, K-contiguous).
    void add(const Desc& Z, const Desc& X, const Desc& Y, int z_buf, int x_buf, int y_buf, int64_t z_base = 0,
             int64_t x_base = 0, int64_t y_base = 0);
    // Same GEMMs over the sectors of Z (sector-major, U(1)), each stored by
    // the epilogue straight into the canonical block list `out` (buffer z_buf).
    // Returns false (and adds nothing) when `out` is not a U(1) canonical list.
    bool add_indirect(const Desc& Z, const Desc& out, const Desc& X, const Desc& Y, int z_buf, int x_buf, int y_buf,
                      int64_t x_base, int64_t y_base);
    void finalize(int variant, int grid);
    void upload(const Allocator& alloc, Deferred* deferred = nullptr);
    hipError_t launch(const PtrTable& bufs, int grid, hipStream_t s) const;
};

// A small contraction as one launch of k_contract_small.
struct SmallProgram {
    std::vector<SmallTask> tasks;
    std::vector<SmallPair> pairs;
    int64_t flops = 0;
    DevMemPtr d_tasks, d_pairs;
    void upload(const Allocator& alloc, Deferred* deferred = nullptr);
    hipError_t launch(const PtrTable& bufs, hipStream_t s) const;
};

struct RecoupleProgram {
    std::vector<FmGroup> groups;
    std::vector<FmBlk> in_blks, out_blks;
    std::vector<double> coef;
    std::vector<FmTask> tasks;
    std::vector<FtGroup> tgroups;   // the same label tuples, for the LDS-tiled kernel
    std::vector<FtTask> ttasks;
    bool tiled = false;             // the permutation moves the input's contiguous (last) leg
    bool tiled_unfit = false;       // a label tuple has more blocks than the tiled kernel takes
    int32_t n_small = 0;            // tasks[0, n_small): tuples of at most kRecoupleSmallN blocks (set by upload)
    int32_t n_tsmall = 0;           // ttasks[0, n_tsmall): tuples of at most kRecoupleTiledSmallN blocks
    int src_dtype = SYM_F32, dst_dtype = SYM_F32;   // element types of the input and the output
    DevMemPtr d_groups, d_in, d_out, d_coef, d_tasks, d_tgroups, d_ttasks;
    // Gamma(tree, perm, tree') of every label tuple; out's leg k is in's leg
    // perm[k]; the tensors start at element in_base / out_base of their
    // buffers.  sign_legs: input legs whose (-1)^(2j) also multiplies the
    // label tuple's coefficients (bit l for leg l)
    void build(const Desc& in, const Desc& out, const std::vector<int32_t>& perm, int64_t in_base = 0,
               int64_t out_base = 0, uint32_t sign_legs = 0);
    // one label tuple: n input and n output block views over dims (output-axis
    // order), gamma[f * n + e]
    void add_group(int rank, const int64_t* dims, const std::vector<FmBlk>& ins, const std::vector<FmBlk>& outs,
                   const std::vector<double>& gamma);
    // a block's view with its strides along the given axes (32-bit checked)
    static FmBlk view(const Block& b, const int32_t* axis, int rank);
    // FUSE of legs leg, leg + 1 of the CHAIN tensor unf into fus (to_fused),
    // or SPLIT of fus back into unf (section "Reshape of indices")
    void build_fuse(const Desc& unf, const Desc& fus, int leg, bool to_fused);
    void upload(const Allocator& alloc, Deferred* deferred = nullptr);
    hipError_t launch(const PtrTable& bufs, int in_buf, int out_buf, hipStream_t s) const;
};

// A device copy of a host table (allocated now; the copy recorded in
// deferred, to be performed in stream order by the caller).
DevMemPtr upload_table(const Allocator& alloc, const std::vector<GemmTile>& v, Deferred* deferred);

// Layout the library uses for its own fused operands.
LayoutOpts workspace_opts(int32_t dtype, bool trans);

// The leg fused from two SU(2) legs of one arrow: every spin c of ja (x) jb,
// degeneracy the sum of da db over the pairs reaching it; inside c the pairs
// run lexicographically (ja, then jb), each over da x db indices row-major.
struct FusedLeg {
    Leg leg;
    std::map<std::array<int32_t, 3>, int64_t> offset;   // (ja, jb, c) -> offset inside c
};
FusedLeg fuse_legs(const Leg& a, const Leg& b);

}  // namespace sym
