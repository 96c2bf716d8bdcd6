// Plan builders: block copies (permute / fuse / split), sector GEMM lists and
// SU(2) recoupling tables.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <map>
#include <numeric>

#include "plan.hpp"

namespace sym {

LayoutOpts workspace_opts(int32_t dtype, bool trans) {
    LayoutOpts o;
    o.trans = trans;
    // rows start on 128-byte cache lines: the GEMM's 64-byte K slices of a
    // row then never straddle two lines (measured 8-20 % faster on the
    // batched BF16 GEMM than 16-byte rows)
    o.ld_align = 128 / static_cast<int64_t>(dtype == SYM_BF16 ? 2 : 4);
    o.base_align = 64;                        // 128/256-byte sector bases
    return o;
}

namespace {

template <typename T>
DevMemPtr upload_vec(const Allocator& alloc, const std::vector<T>& v, Deferred* deferred = nullptr) {
    if (v.empty()) return nullptr;
    DevMemPtr m = alloc(v.size() * sizeof(T));
    if (deferred) {
        deferred->push_back({m->ptr, v.data(), v.size() * sizeof(T)});
        return m;
    }
    hipError_t e = hipMemcpy(m->ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) throw Error(SYM_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// CopyProgram
// ---------------------------------------------------------------------------

// Division by an invariant divisor for dividends below 2^31: with
// s = ceil(log2 d) and m = ceil(2^(31+s) / d) < 2^32, the error of n m / 2^(31+s)
// against n / d is below n (m d - 2^(31+s)) / (d 2^(31+s)) < 2^-s <= 1/d, too
// small to move the floor (round-up multiplier method, Granlund and
// Montgomery, PLDI 1994).
// Round-up multiplier m = ceil(2^(31+s) / v), s = ceil(log2 v): then
// floor(x / v) = (x m) >> (31 + s) for every 0 <= x < 2^31.
static void magic_divisor(int32_t divisor, uint32_t& mag, int32_t& shf) {
    const uint64_t v = static_cast<uint64_t>(std::max(1, divisor));
    int s = 0;
    while ((uint64_t{1} << s) < v) ++s;
    const uint64_t m = ((uint64_t{1} << (31 + s)) + v - 1) / v;
    if (m >= (uint64_t{1} << 32)) throw Error(SYM_E_UNSUPPORTED, "division multiplier out of range");
    mag = static_cast<uint32_t>(m);
    shf = s;
}

static void set_divisor(CopyOp& op, int d) {
    uint32_t m;
    int32_t s;
    magic_divisor(op.size[d], m, s);
    op.mag[d] = m;
    op.shf[d] = s;
}

void CopyProgram::add(const Desc& src, const Desc& dst, const std::vector<int32_t>& perm, int src_buf, int dst_buf,
                      int64_t src_base, int64_t dst_base) {
    const int rank = dst.rank;
    if (src.rank != rank || static_cast<int>(perm.size()) != rank) throw Error(SYM_E_ARG, "permutation rank mismatch");
    int32_t lab[SYM_MAX_RANK];
    for (const Block& b : dst.blocks) {
        for (int i = 0; i < rank; ++i) lab[perm[static_cast<size_t>(i)]] = b.labels[static_cast<size_t>(i)];
        if (src.tree != dst.tree) throw Error(SYM_E_ARG, "block copies keep the SU(2) tree");
        const int32_t si = src.find_block(lab, b);
        if (si < 0) throw Error(SYM_E_MISMATCH, "destination block has no source block");
        const Block& sb = src.blocks[static_cast<size_t>(si)];
        // dims in destination leg order, outermost first
        int64_t sz[SYM_MAX_RANK], ss[SYM_MAX_RANK], ds[SYM_MAX_RANK];
        int nd = 0;
        for (int i = 0; i < rank; ++i) {
            if (b.shape[static_cast<size_t>(i)] == 1) continue;
            sz[nd] = b.shape[static_cast<size_t>(i)];
            ss[nd] = sb.stride[static_cast<size_t>(perm[static_cast<size_t>(i)])];
            ds[nd] = b.stride[static_cast<size_t>(i)];
            ++nd;
        }
        // merge an outer dim into the next inner one when both sides are contiguous across them
        int64_t msz[SYM_MAX_RANK], mss[SYM_MAX_RANK], mds[SYM_MAX_RANK];
        int m = 0;
        for (int i = nd - 1; i >= 0; --i) {
            if (m > 0 && ss[i] == mss[m - 1] * msz[m - 1] && ds[i] == mds[m - 1] * msz[m - 1]) {
                msz[m - 1] *= sz[i];
            } else {
                msz[m] = sz[i];
                mss[m] = ss[i];
                mds[m] = ds[i];
                ++m;
            }
        }
        if (m == 0) {
            msz[0] = 1;
            mss[0] = 1;
            mds[0] = 1;
            m = 1;
        }
        if (m > kMaxCopyDims) throw Error(SYM_E_UNSUPPORTED, "block copy needs more than 6 strided dims");
        if (b.size > INT32_MAX) throw Error(SYM_E_UNSUPPORTED, "block exceeds 2^31 elements");
        // innermost = the destination's most contiguous dim, so that lanes write
        // consecutive addresses (any order of the index space is valid)
        int ord[SYM_MAX_RANK];
        for (int k = 0; k < m; ++k) ord[k] = k;
        std::stable_sort(ord, ord + m, [&](int x, int y) { return mds[x] < mds[y]; });
        CopyOp op{};
        op.src_off = src_base + sb.offset;
        op.dst_off = dst_base + b.offset;
        for (int d = 0; d < kMaxCopyDims; ++d) {
            op.size[d] = 1;
            op.sstride[d] = 0;
            op.dstride[d] = 0;
        }
        for (int k = 0; k < m; ++k) {
            const int d = kMaxCopyDims - 1 - k;
            op.size[d] = static_cast<int32_t>(msz[ord[k]]);
            op.sstride[d] = mss[ord[k]];
            op.dstride[d] = mds[ord[k]];
        }
        for (int d = 0; d < kMaxCopyDims; ++d) set_divisor(op, d);
        // fermion parity: R(1,1->0) = -1 for every pair of odd legs whose
        // order the permutation reverses (dst leg i is src leg perm[i])
        op.neg = 0;
        if (src.group == SYM_Z2F)
            for (int i = 0; i < rank; ++i)
                for (int j = i + 1; j < rank; ++j)
                    if (perm[static_cast<size_t>(i)] > perm[static_cast<size_t>(j)] &&
                        (b.labels[static_cast<size_t>(i)] & 1) && (b.labels[static_cast<size_t>(j)] & 1))
                        op.neg ^= 1;
        op.ndim = m;
        op.count = static_cast<int32_t>(b.size);
        op.src_buf = src_buf;
        op.dst_buf = dst_buf;
        op.tj = -1;
        op.ihi = op.jhi = -1;
        op.src_len = src_base + src.numel;
        // rows of one contiguous source run, written along contiguous destination rows
        constexpr int II = kMaxCopyDims - 1;
        op.rowcopy = (m <= 2 && op.sstride[II] == 1 && op.dstride[II] == 1 &&
                      (m == 1 || op.sstride[II - 1] == op.size[II]))
                         ? 1
                         : 0;
        // a transposing copy (the source is contiguous along another dim) goes
        // through the LDS-tiled kernel when both dims are wide enough
        constexpr int I = kMaxCopyDims - 1;
        if (m >= 2 && op.sstride[I] != 1 && op.size[I] >= 4) {
            for (int d = kMaxCopyDims - 2; d >= kMaxCopyDims - m; --d)
                if (op.sstride[d] == 1 && op.size[d] >= 4) op.tj = d;
        }
        ops.push_back(op);
    }
}

void CopyProgram::finalize() {
    constexpr int32_t kChunk = 4096;     // elements per task
    constexpr int64_t kPerWg = 4096;     // elements a workgroup aims for
    constexpr int32_t kMaxTasksPerWg = 64;
    tasks.clear();
    wg_begin.clear();
    tile_tasks.clear();
    vtile_tasks.clear();
    mtile_tasks.clear();
    row_tasks.clear();
    for (size_t i = 0; i < ops.size(); ++i) {
        CopyOp& op = ops[i];
        if (op.tj >= 0) {
            constexpr int I = kMaxCopyDims - 1;
            // destination rows of unit stride take the vectorized kernel, as
            // long as one tile's source rows span less than 2^29 bytes
            const int esz = src_dtype == SYM_BF16 ? 2 : 4;
            const int ti = vtile_rows(esz);
            const int tc = vtile_cols(esz);
            const bool vec = op.dstride[I] == 1 && op.sstride[I] > 0 && op.sstride[I] * ti * esz < (int64_t{1} << 29);
            op.ihi = op.jhi = -1;
            if (vec && static_cast<int64_t>(op.count) * esz < (int64_t{1} << 29)) {
                // small blocks: continue a short row dim with the dim that
                // follows it in the destination, a short column dim with the
                // one that follows it in the source, so tiles fill up (the
                // block spans less than 2^29 bytes, so any tile does too)
                for (int d = kMaxCopyDims - 2; d >= kMaxCopyDims - op.ndim; --d) {
                    if (d == op.tj) continue;
                    if (op.ihi < 0 && op.size[I] < ti && op.dstride[d] == op.size[I]) op.ihi = d;
                    else if (op.jhi < 0 && op.size[op.tj] < tc && op.sstride[d] == op.size[op.tj]) op.jhi = d;
                }
            }
            int64_t outer = 1;
            for (int d = kMaxCopyDims - 2; d >= kMaxCopyDims - op.ndim; --d)
                if (d != op.tj && d != op.ihi && d != op.jhi) outer *= op.size[d];
            const int64_t nI = static_cast<int64_t>(op.size[I]) * (op.ihi >= 0 ? op.size[op.ihi] : 1);
            const int64_t nJ = static_cast<int64_t>(op.size[op.tj]) * (op.jhi >= 0 ? op.size[op.jhi] : 1);
            const int cj = vec ? tc : kTile;
            const int nj = static_cast<int>((nJ + cj - 1) / cj);
            const int ni = static_cast<int>((nI + (vec ? ti : kTile) - 1) / (vec ? ti : kTile));
            if (vec && op.ihi < 0 && op.jhi < 0 && op.count >= kChunk &&
                4 * nI * nJ < static_cast<int64_t>(ti) * tc) {
                // a small transpose that fills under a quarter of a tile and
                // has no dim to merge: element-wise (the rows sit in L2).
                // Blocks below one element-wise task stay tiled: the
                // element-wise kernel runs a workgroup's tasks one after the
                // other, which a contraction of tiny blocks would wait for.
                for (int32_t s0 = 0; s0 < op.count; s0 += kChunk)
                    tasks.push_back({static_cast<int32_t>(i), s0, std::min(kChunk, op.count - s0), 0});
                continue;
            }
            std::vector<TileTask>& list =
                !vec ? tile_tasks : (op.ihi >= 0 || op.jhi >= 0) ? mtile_tasks : vtile_tasks;
            // tiles adjacent along the source's contiguous dim share the
            // cache lines at their boundary: keep them next to each other
            for (int64_t o = 0; o < outer; ++o)
                for (int it = 0; it < ni; ++it)
                    for (int jt = 0; jt < nj; ++jt)
                        list.push_back({static_cast<int32_t>(i), static_cast<int32_t>(o), jt, it});
            continue;
        }
        if (op.rowcopy) {
            constexpr int II = kMaxCopyDims - 1;
            const int32_t L = op.size[II], R = op.ndim > 1 ? op.size[II - 1] : 1;
            if (L <= kRowStage) {
                const int32_t per = std::max<int32_t>(1, kRowStage / L);
                for (int32_t r = 0; r < R; r += per)
                    row_tasks.push_back({static_cast<int32_t>(i), r, std::min(per, R - r), 0, L, 0, 0, 0});
            } else {
                for (int32_t r = 0; r < R; ++r)
                    for (int32_t c = 0; c < L; c += kRowStage)
                        row_tasks.push_back({static_cast<int32_t>(i), r, 1, c, std::min(kRowStage, L - c), 0, 0, 0});
            }
            continue;
        }
        for (int32_t s = 0; s < op.count; s += kChunk)
            tasks.push_back({static_cast<int32_t>(i), s, std::min(kChunk, op.count - s), 0});
    }
    wg_begin.push_back(0);
    int64_t acc = 0;
    int32_t n_in = 0;
    for (size_t t = 0; t < tasks.size(); ++t) {
        acc += tasks[t].count;
        ++n_in;
        if (acc >= kPerWg || n_in >= kMaxTasksPerWg) {
            wg_begin.push_back(static_cast<int32_t>(t + 1));
            acc = 0;
            n_in = 0;
        }
    }
    if (wg_begin.back() != static_cast<int32_t>(tasks.size())) wg_begin.push_back(static_cast<int32_t>(tasks.size()));
    // The tiled kernel runs tile_grid workgroups; workgroup w sits on XCD
    // w % 8 and takes tasks w, w + tile_grid, ...  Each round of tile_grid
    // tasks gives every XCD a contiguous run of the sequence, so that tiles
    // sharing boundary lines meet in the same L2.
    tile_grid = xcd_order(tile_tasks);
    vtile_grid = xcd_order(vtile_tasks);
    mtile_grid = xcd_order(mtile_tasks);
}

int32_t CopyProgram::xcd_order(std::vector<TileTask>& list) {
    const int64_t n = static_cast<int64_t>(list.size());
    int32_t grid = static_cast<int32_t>(std::min<int64_t>(n, kTileGridMax));
    if (grid >= 8) {
        const int64_t g = grid - grid % 8, per = g / 8;
        grid = static_cast<int32_t>(g);
        std::vector<TileTask> seq(list);
        for (int64_t r0 = 0; r0 + g <= n; r0 += g)
            for (int64_t w = 0; w < g; ++w)
                list[static_cast<size_t>(r0 + w)] = seq[static_cast<size_t>(r0 + (w % 8) * per + w / 8)];
    }
    return grid;
}

void CopyProgram::upload(const Allocator& alloc, Deferred* deferred) {
    d_ops = upload_vec(alloc, ops, deferred);
    d_tasks = upload_vec(alloc, tasks, deferred);
    d_wg = upload_vec(alloc, wg_begin, deferred);
    d_tile_tasks = upload_vec(alloc, tile_tasks, deferred);
    d_row_tasks = upload_vec(alloc, row_tasks, deferred);
    d_vtile_tasks = upload_vec(alloc, vtile_tasks, deferred);
    d_mtile_tasks = upload_vec(alloc, mtile_tasks, deferred);
}

hipError_t CopyProgram::launch(const PtrTable& bufs, hipStream_t s) const {
    if (ops.empty()) return hipSuccess;
    if (!tasks.empty()) {
        hipError_t e = launch_permute(src_dtype, dst_dtype, static_cast<const CopyOp*>(d_ops->ptr),
                                      static_cast<const CopyTask*>(d_tasks->ptr), static_cast<const int32_t*>(d_wg->ptr),
                                      static_cast<int32_t>(wg_begin.size()) - 1, bufs, s);
        if (e != hipSuccess) return e;
    }
    if (!row_tasks.empty()) {
        const int32_t n = static_cast<int32_t>(row_tasks.size());
        hipError_t e = launch_copy_rows(src_dtype, dst_dtype, static_cast<const CopyOp*>(d_ops->ptr),
                                        static_cast<const RowTask*>(d_row_tasks->ptr), n,
                                        std::min<int32_t>(n, kTileGridMax), bufs, s);
        if (e != hipSuccess) return e;
    }
    if (!vtile_tasks.empty()) {
        hipError_t e = launch_transpose_vec(src_dtype, dst_dtype, false, static_cast<const CopyOp*>(d_ops->ptr),
                                            static_cast<const TileTask*>(d_vtile_tasks->ptr),
                                            static_cast<int32_t>(vtile_tasks.size()), vtile_grid, bufs, s);
        if (e != hipSuccess) return e;
    }
    if (!mtile_tasks.empty()) {
        hipError_t e = launch_transpose_vec(src_dtype, dst_dtype, true, static_cast<const CopyOp*>(d_ops->ptr),
                                            static_cast<const TileTask*>(d_mtile_tasks->ptr),
                                            static_cast<int32_t>(mtile_tasks.size()), mtile_grid, bufs, s);
        if (e != hipSuccess) return e;
    }
    if (!tile_tasks.empty())
        return launch_permute_tiled(src_dtype, dst_dtype, static_cast<const CopyOp*>(d_ops->ptr),
                                    static_cast<const TileTask*>(d_tile_tasks->ptr),
                                    static_cast<int32_t>(tile_tasks.size()), tile_grid, bufs, s);
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// GemmProgram
// ---------------------------------------------------------------------------

namespace {

// GEMM view of a sector: outer tuples (matrix rows as stored) and inner
// tuples (the contiguous dimension).
struct View {
    const std::vector<Tuple>* outer;
    const std::vector<Tuple>* inner;
    int64_t n_outer, n_inner, ld, offset;
};

View view_of(const Desc& d, const Sector& s) {
    if (d.opts.trans) return {&s.col_tuples, &s.row_tuples, s.cols, s.rows, s.ld, s.offset};
    return {&s.row_tuples, &s.col_tuples, s.rows, s.cols, s.ld, s.offset};
}

bool same_tuples(const std::vector<Tuple>& a, const std::vector<Tuple>& b) {
    if (a.size() != b.size()) return false;
    for (size_t i = 0; i < a.size(); ++i)
        if (!(a[i] == b[i]) || a[i].dim != b[i].dim) return false;
    return true;
}

// sector index of each outer tuple (U(1): a tuple lies in one sector).
std::unordered_map<std::string, int32_t> outer_index(const Desc& d) {
    std::unordered_map<std::string, int32_t> m;
    for (size_t si = 0; si < d.sectors.size(); ++si) {
        View v = view_of(d, d.sectors[si]);
        for (const Tuple& t : *v.outer) m[label_key(t.lab.data(), t.n, 0)] = static_cast<int32_t>(si);
    }
    return m;
}

}  // namespace

void GemmProgram::add(const Desc& Z, const Desc& X, const Desc& Y, int z_buf, int x_buf, int y_buf, int64_t z_base,
                      int64_t x_base, int64_t y_base) {
    if (Z.opts.trans) throw Error(SYM_E_UNSUPPORTED, "GEMM output must not be transposed");
    const bool su2 = Z.group == SYM_SU2;
    std::unordered_map<std::string, int32_t> xi, yi;
    if (!su2) {
        xi = outer_index(X);
        yi = outer_index(Y);
    }
    for (const Sector& zs : Z.sectors) {
        GemmProb p{};
        p.M = static_cast<int32_t>(zs.rows);
        p.N = static_cast<int32_t>(zs.cols);
        p.c_off = z_base + zs.offset;
        p.ldc = static_cast<int32_t>(zs.ld);
        p.c_buf = z_buf;
        p.a_buf = x_buf;
        p.b_buf = y_buf;
        p.lda = p.ldb = 1;
        p.K = 0;
        int32_t xs = -1, ys = -1;
        if (su2) {
            xs = X.find_sector(zs.label);
            ys = Y.find_sector(zs.label);
        } else {
            if (zs.row_tuples.empty() || zs.col_tuples.empty()) continue;
            auto a = xi.find(label_key(zs.row_tuples[0].lab.data(), zs.row_tuples[0].n, 0));
            auto b = yi.find(label_key(zs.col_tuples[0].lab.data(), zs.col_tuples[0].n, 0));
            if (a != xi.end()) xs = a->second;
            if (b != yi.end()) ys = b->second;
        }
        if (xs >= 0 && ys >= 0) {
            View xv = view_of(X, X.sectors[static_cast<size_t>(xs)]);
            View yv = view_of(Y, Y.sectors[static_cast<size_t>(ys)]);
            if (!same_tuples(*xv.outer, zs.row_tuples) || !same_tuples(*yv.outer, zs.col_tuples))
                throw Error(SYM_E_MISMATCH, "operand sectors do not line up with the output sector");
            if (!same_tuples(*xv.inner, *yv.inner))
                throw Error(SYM_E_MISMATCH, "contracted tuples differ between the operands");
            p.K = static_cast<int32_t>(xv.n_inner);
            p.a_off = x_base + xv.offset;
            p.b_off = y_base + yv.offset;
            p.lda = static_cast<int32_t>(xv.ld);
            p.ldb = static_cast<int32_t>(yv.ld);
        }
        if (zs.rows > INT32_MAX || zs.cols > INT32_MAX) throw Error(SYM_E_UNSUPPORTED, "sector too large");
        flops += 2 * static_cast<int64_t>(p.M) * p.N * p.K;
        probs.push_back(p);
    }
}

bool GemmProgram::add_indirect(const Desc& Z, const Desc& out, const Desc& X, const Desc& Y, int z_buf, int x_buf,
                               int y_buf, int64_t x_base, int64_t y_base) {
    if (!is_abelian(Z.group) || out.group != Z.group || out.n_row != out.rank || out.opts.trans ||
        out.dtype != SYM_F32 || out.legs != Z.legs || out.qtot != Z.qtot || Z.opts.trans)
        return false;
    // 32-bit address terms, 24-bit factors (see EpiRow)
    constexpr int64_t k24 = int64_t{1} << 24;
    if (out.numel >= (int64_t{1} << 29)) return false;   // byte offsets below 2^31
    for (const Sector& zs : Z.sectors) {
        if (zs.cols >= k24) return false;
        for (const Tuple& t : zs.row_tuples)
            if (t.dim >= k24) return false;
        for (const Tuple& t : zs.col_tuples)
            if (t.dim >= k24) return false;
    }
    // check the address formula against every block before committing
    const size_t p0 = probs.size();
    std::vector<EpiRow> rows_add;
    std::vector<EpiCol> cols_add;
    std::vector<int64_t> ri(Z.sectors.size()), ci(Z.sectors.size());
    int32_t lab[SYM_MAX_RANK];
    for (size_t si = 0; si < Z.sectors.size(); ++si) {
        const Sector& zs = Z.sectors[si];
        ri[si] = static_cast<int64_t>(erows.size() + rows_add.size());
        ci[si] = static_cast<int64_t>(ecols.size() + cols_add.size());
        const int nr = Z.n_row, nc = Z.rank - Z.n_row;
        for (size_t r = 0; r < zs.row_tuples.size(); ++r) {
            const Tuple& rt = zs.row_tuples[r];
            int64_t base = -1;
            for (size_t c = 0; c < zs.col_tuples.size(); ++c) {
                const Tuple& ct = zs.col_tuples[c];
                for (int l = 0; l < nr; ++l) lab[l] = rt.lab[static_cast<size_t>(l)];
                for (int l = 0; l < nc; ++l) lab[nr + l] = ct.lab[static_cast<size_t>(l)];
                const int32_t bi = out.find_block(lab, -1);
                if (bi < 0) return false;
                const int64_t off = out.blocks[static_cast<size_t>(bi)].offset;
                if (c == 0) base = off;
                if (off != base + rt.dim * zs.col_off[c]) return false;
            }
            for (int64_t t = 0; t < rt.dim; ++t)
                rows_add.push_back({static_cast<int32_t>(base), static_cast<int32_t>(t), static_cast<int32_t>(rt.dim), 0});
        }
        for (size_t c = 0; c < zs.col_tuples.size(); ++c) {
            const Tuple& ct = zs.col_tuples[c];
            for (int64_t t = 0; t < ct.dim; ++t)
                cols_add.push_back({static_cast<int32_t>(zs.col_off[c]), static_cast<int32_t>(t), static_cast<int32_t>(ct.dim), 0});
        }
    }
    add(Z, X, Y, z_buf, x_buf, y_buf, 0, x_base, y_base);
    if (probs.size() - p0 != Z.sectors.size()) throw Error(SYM_E_MISMATCH, "indirect GEMM sector count");
    for (size_t si = 0; si < Z.sectors.size(); ++si) {
        GemmProb& p = probs[p0 + si];
        p.indirect = 1;
        p.c_off = 0;
        p.ri_off = ri[si];
        p.ci_off = ci[si];
    }
    erows.insert(erows.end(), rows_add.begin(), rows_add.end());
    ecols.insert(ecols.end(), cols_add.begin(), cols_add.end());
    return true;
}

void GemmProgram::finalize(int v, int grid) {
    if (gemm_variant_direct(compute, v)) {
        // direct-load kernels address a tile's rows through a 32-bit range
        for (const GemmProb& p : probs)
            if (p.lda >= gemm_direct_max_ld() || p.ldb >= gemm_direct_max_ld()) {
                v = gemm_default_variant_wide(compute);
                break;
            }
    }
    variant = v;
    const GemmVariant gv = gemm_variant(compute, v);
    // longest-processing-time order: all tiles of one sector cost ~K, so sort
    // sectors by K (then size) descending and emit their tiles together.
    std::vector<int32_t> order(probs.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const GemmProb& x = probs[static_cast<size_t>(a)];
        const GemmProb& y = probs[static_cast<size_t>(b)];
        if (x.K != y.K) return x.K > y.K;
        return static_cast<int64_t>(x.M) * x.N > static_cast<int64_t>(y.M) * y.N;
    });
    // inside a sector, walk tiles in groups of kGroupM tile rows, column by
    // column, so that consecutive tiles share A row panels and B column panels
    constexpr int kGroupM = 8;
    std::vector<GemmTile> seq;
    for (int32_t pi : order) {
        const GemmProb& p = probs[static_cast<size_t>(pi)];
        const int tm = (p.M + gv.mt - 1) / gv.mt, tn = (p.N + gv.nt - 1) / gv.nt;
        for (int g0 = 0; g0 < tm; g0 += kGroupM)
            for (int j = 0; j < tn; ++j)
                for (int i = g0; i < std::min(tm, g0 + kGroupM); ++i) seq.push_back({pi, i, j, 0});
    }
    // The persistent grid runs `grid` workgroups; workgroup w sits on XCD
    // w % 8 and takes tiles w, w + grid, ...  Give each XCD a contiguous run
    // of the sequence per round, so that the tiles one XCD holds at a time
    // share its L2.  (Putting the XCDs out of phase, so that they write their
    // C tiles at different times, measured no faster.)
    tiles.assign(seq.size(), GemmTile{});
    const int64_t g = std::max(8, grid - grid % 8);
    const int64_t n = static_cast<int64_t>(seq.size());
    const int64_t per = g / 8;
    for (int64_t r0 = 0; r0 < n; r0 += g) {
        const int64_t len = std::min(g, n - r0);
        if (len < g) {
            for (int64_t k = 0; k < len; ++k) tiles[static_cast<size_t>(r0 + k)] = seq[static_cast<size_t>(r0 + k)];
            break;
        }
        for (int64_t w = 0; w < g; ++w)
            tiles[static_cast<size_t>(r0 + w)] = seq[static_cast<size_t>(r0 + (w % 8) * per + w / 8)];
    }
}

void SmallProgram::upload(const Allocator& alloc, Deferred* deferred) {
    d_tasks = upload_vec(alloc, tasks, deferred);
    d_pairs = upload_vec(alloc, pairs, deferred);
}

hipError_t SmallProgram::launch(const PtrTable& bufs, hipStream_t s) const {
    if (tasks.empty()) return hipSuccess;
    return launch_contract_small(static_cast<const SmallTask*>(d_tasks->ptr), static_cast<int32_t>(tasks.size()),
                                 d_pairs ? static_cast<const SmallPair*>(d_pairs->ptr) : nullptr, bufs, s);
}

DevMemPtr upload_table(const Allocator& alloc, const std::vector<GemmTile>& v, Deferred* deferred) {
    return upload_vec(alloc, v, deferred);
}

void GemmProgram::upload(const Allocator& alloc, Deferred* deferred) {
    d_probs = upload_vec(alloc, probs, deferred);
    d_tiles = upload_vec(alloc, tiles, deferred);
    d_rows = upload_vec(alloc, erows, deferred);
    d_cols = upload_vec(alloc, ecols, deferred);
}

hipError_t GemmProgram::launch(const PtrTable& bufs, int grid, hipStream_t s) const {
    if (tiles.empty()) return hipSuccess;
    const int g = std::max(1, std::min(grid, static_cast<int>(tiles.size())));
    return launch_gemm(compute, variant, static_cast<const GemmProb*>(d_probs->ptr),
                       static_cast<const GemmTile*>(d_tiles->ptr), static_cast<int32_t>(tiles.size()), g,
                       d_rows ? static_cast<const EpiRow*>(d_rows->ptr) : nullptr,
                       d_cols ? static_cast<const EpiCol*>(d_cols->ptr) : nullptr, bufs, s);
}

// ---------------------------------------------------------------------------
// RecoupleProgram: LEFT tree (legs 1,2,3,4) -> RIGHT tree on legs (1,3,2,4)
// ---------------------------------------------------------------------------

namespace {

int64_t isqrt64(int64_t x) {
    int64_t r = 0;
    while ((r + 1) * (r + 1) <= x) ++r;
    return r;
}

// Box of the tiled recoupling kernel for one label tuple (see FtGroup): the
// axis fixed per task is output axis 0, or axis 1 when the input is
// contiguous along output axis 0; the box holds kFtElems / n entries of each
// block, shaped so that both the input runs (along the tile axis of smallest
// input stride) and the output runs (along the innermost axes) are long.
void choose_box(FtGroup& g, const FmBlk& in0) {
    int fastest = -1;
    for (int k = 0; k < 4; ++k)
        if (g.dim[k] > 1 && (fastest < 0 || in0.stride[k] < in0.stride[fastest] ||
                             (in0.stride[k] == in0.stride[fastest] && k > fastest)))
            fastest = k;
    g.ax[0] = fastest == 0 ? 1 : 0;
    for (int k = 0, s = 1; k < 4; ++k)
        if (k != g.ax[0]) g.ax[s++] = k;
    int64_t D[4] = {1, g.dim[g.ax[1]], g.dim[g.ax[2]], g.dim[g.ax[3]]};
    // load order: tile slots by input stride (size-1 axes last, ties to the inner slot)
    int slot[3] = {1, 2, 3};
    std::sort(slot, slot + 3, [&](int x, int y) {
        const int64_t sx = D[x] == 1 ? INT64_MAX : in0.stride[g.ax[x]];
        const int64_t sy = D[y] == 1 ? INT64_MAX : in0.stride[g.ax[y]];
        if (sx != sy) return sx < sy;
        return x > y;
    });
    for (int k = 0; k < 3; ++k) g.ld[k] = slot[k];
    const int64_t E = std::max<int64_t>(1, kFtElems / g.n);
    int64_t T[4] = {1, 1, 1, 1};
    const int f = slot[0], m = slot[1];
    if (f == 3) {
        // the input keeps the output's innermost axis: runs along slot 3, then
        // along the slot whose input stride comes next
        T[3] = std::min(D[3], E);
        const int64_t rem = std::max<int64_t>(1, E / T[3]);
        if (m == 2) {
            T[2] = std::min(D[2], rem);
            T[1] = std::min(D[1], std::max<int64_t>(1, rem / T[2]));
        } else {
            T[2] = std::min(D[2], std::max<int64_t>(1, isqrt64(rem)));
            T[1] = std::min(D[1], std::max<int64_t>(1, rem / T[2]));
            if (T[1] == D[1]) T[2] = std::min(D[2], std::max<int64_t>(1, rem / T[1]));
        }
    } else {
        // a transpose between the input's contiguous slot f and slot 3
        T[3] = std::min(D[3], std::max<int64_t>(16, isqrt64(E)));
        const int64_t rem = std::max<int64_t>(1, E / T[3]);
        T[f] = std::min(D[f], rem);
        const int o = 6 - 3 - f;   // the remaining slot
        T[o] = std::min(D[o], std::max<int64_t>(1, rem / T[f]));
    }
    g.t[0] = 1;
    for (int k = 1; k < 4; ++k) g.t[k] = static_cast<int32_t>(T[k]);
    g.esz = g.t[1] * g.t[2] * g.t[3];
    if (static_cast<int64_t>(g.esz) * g.n > kFtElems) throw Error(SYM_E_UNSUPPORTED, "recoupling box too large");
    const int32_t divs[5] = {g.t[3], g.t[2], g.t[g.ld[0]], g.t[g.ld[1]], g.esz};
    for (int k = 0; k < 5; ++k) magic_divisor(divs[k], g.mag[k], g.shf[k]);
}

}  // namespace

FmBlk RecoupleProgram::view(const Block& b, const int32_t* axis, int rank) {
    FmBlk fb{};
    fb.off = b.offset;
    int64_t span = 0;
    for (int l = 0; l < rank; ++l) {
        const int64_t st = b.stride[static_cast<size_t>(axis[l])];
        span += (b.shape[static_cast<size_t>(axis[l])] - 1) * st;
        if (st < 0 || st >= (int64_t{1} << 31)) throw Error(SYM_E_UNSUPPORTED, "block stride beyond 32 bits");
        fb.stride[l] = static_cast<int32_t>(st);
    }
    if (span >= (int64_t{1} << 31)) throw Error(SYM_E_UNSUPPORTED, "block span beyond 32 bits");
    return fb;
}

void RecoupleProgram::add_group(int rank, const int64_t* dims, const std::vector<FmBlk>& ins,
                                const std::vector<FmBlk>& outs, const std::vector<double>& gamma) {
    const int n = static_cast<int>(ins.size());
    if (static_cast<int>(outs.size()) != n || gamma.size() != static_cast<size_t>(n) * n)
        throw Error(SYM_E_MISMATCH, "recoupling group is not square");
    if (n > kMaxRecouple) throw Error(SYM_E_UNSUPPORTED, "too many blocks in one label tuple (above 32)");
    if (rank > kMaxRecoupleRank) throw Error(SYM_E_UNSUPPORTED, "rank above 8");
    FmGroup g{};
    g.n = n;
    g.rank = rank;
    int64_t elems = 1;
    for (int k = 0; k < kMaxRecoupleRank; ++k) {
        g.d[k] = k < rank ? static_cast<int32_t>(dims[k]) : 1;
        magic_divisor(g.d[k], g.mag[k], g.shf[k]);
        elems *= g.d[k];
    }
    if (elems >= (int64_t{1} << 31)) throw Error(SYM_E_UNSUPPORTED, "block too large to recouple");
    g.in_first = static_cast<int32_t>(in_blks.size());
    g.out_first = static_cast<int32_t>(out_blks.size());
    g.coef_first = static_cast<int32_t>(coef.size());
    g.same_in = g.same_out = 1;
    for (int i = 0; i < n; ++i)
        for (int l = 0; l < rank; ++l) {
            g.same_in &= ins[static_cast<size_t>(i)].stride[l] == ins[0].stride[l];
            g.same_out &= outs[static_cast<size_t>(i)].stride[l] == outs[0].stride[l];
        }
    in_blks.insert(in_blks.end(), ins.begin(), ins.end());
    out_blks.insert(out_blks.end(), outs.begin(), outs.end());
    coef.insert(coef.end(), gamma.begin(), gamma.end());
    if (rank == 4 && n > kMaxRecoupleTiled) tiled_unfit = true;
    if (rank == 4 && n <= kMaxRecoupleTiled) {
        FtGroup tg{};
        tg.n = n;
        for (int k = 0; k < 4; ++k) tg.dim[k] = g.d[k];
        tg.in_first = g.in_first;
        tg.out_first = g.out_first;
        tg.coef_first = g.coef_first;
        choose_box(tg, ins[0]);
        const int32_t tgi = static_cast<int32_t>(tgroups.size());
        for (int32_t o0 = 0; o0 < tg.dim[tg.ax[0]]; ++o0)
            for (int32_t o1 = 0; o1 < tg.dim[tg.ax[1]]; o1 += tg.t[1])
                for (int32_t o2 = 0; o2 < tg.dim[tg.ax[2]]; o2 += tg.t[2])
                    for (int32_t o3 = 0; o3 < tg.dim[tg.ax[3]]; o3 += tg.t[3])
                        ttasks.push_back({tgi, {o0, o1, o2, o3}, {0, 0, 0}});
        tgroups.push_back(tg);
    }
    for (int64_t st = 0; st < elems; st += kRecoupleChunk)
        tasks.push_back({static_cast<int32_t>(groups.size()), static_cast<int32_t>(st),
                         static_cast<int32_t>(std::min<int64_t>(kRecoupleChunk, elems - st)), 0});
    groups.push_back(g);
}

namespace {

// the CHAIN key of a block of a CHAIN, OPERATOR or LEFT tensor (the rank-4
// trees list their one intermediate spin, which is the CHAIN key there)
std::vector<int32_t> key_of(const Desc& d, const Block& b) {
    if (d.tree == SYM_TREE_CHAIN) return std::vector<int32_t>(b.inner.begin(), b.inner.begin() + b.n_inner);
    return std::vector<int32_t>{b.internal};
}

int32_t find_keyed(const Desc& d, const int32_t* labels, const std::vector<int32_t>& key) {
    if (d.tree == SYM_TREE_CHAIN) return d.find_block_inner(labels, key.data(), static_cast<int32_t>(key.size()));
    if (key.size() != 1) return -1;
    return d.find_block(labels, key[0]);
}

bool chain_like(const Desc& d) {
    return d.tree == SYM_TREE_CHAIN || d.tree == SYM_TREE_OPERATOR || d.tree == SYM_TREE_LEFT;
}

}  // namespace

void RecoupleProgram::build(const Desc& in, const Desc& out, const std::vector<int32_t>& perm, int64_t in_base,
                            int64_t out_base, uint32_t sign_legs) {
    // (-1)^(2j) summed over the marked legs of a label tuple (doubled spins)
    auto tuple_sign = [&](const int32_t* labels, std::vector<double>& gamma) {
        int32_t s = 0;
        for (int l = 0; l < in.rank; ++l)
            if (sign_legs >> l & 1u) s += labels[l];
        if (s & 1)
            for (double& g : gamma) g = -g;
    };
    if (in.group != SYM_SU2 || out.group != SYM_SU2 || in.rank != out.rank || static_cast<int>(perm.size()) != in.rank)
        throw Error(SYM_E_UNSUPPORTED, "recoupling acts on SU(2) tensors of equal rank");
    src_dtype = in.dtype;
    dst_dtype = out.dtype;
    if (!recouple_dtypes_supported(src_dtype, dst_dtype))
        throw Error(SYM_E_DTYPE, "recoupling takes F32 -> F32, F32 -> BF16 or BF16 -> BF16");
    const int rank = in.rank;
    // Inputs are row-major over their legs in every layout, so the input is
    // contiguous along its last leg.  When that leg stays last the
    // element-wise kernel reads and writes along the same runs (measured
    // 2.7-3.0 TB/s on config 5, slightly ahead of the tiled kernel); when it
    // moves, the tiled kernel (rank 4) transposes through LDS (full reversal:
    // 2.5 against 0.73 TB/s).
    tiled = rank == 4 && perm[static_cast<size_t>(rank - 1)] != rank - 1;
    tiled_unfit = false;
    int64_t dims[kMaxRecoupleRank];
    if (in.tree == SYM_TREE_CHAIN || out.tree == SYM_TREE_CHAIN) {
        if (!chain_like(in) || !chain_like(out))
            throw Error(SYM_E_UNSUPPORTED, "CHAIN recoupling takes CHAIN, OPERATOR or LEFT tensors");
        std::vector<int32_t> ain, aout;
        for (const Leg& l : in.legs) ain.push_back(l.arrow);
        for (const Leg& l : out.legs) aout.push_back(l.arrow);
        std::vector<std::vector<int32_t>> ki, ko;
        std::vector<double> gamma;
        size_t i = 0;
        while (i < in.blocks.size()) {
            const Block& b0 = in.blocks[i];
            size_t jend = i;
            while (jend < in.blocks.size() &&
                   std::equal(in.blocks[jend].labels.begin(), in.blocks[jend].labels.begin() + rank, b0.labels.begin()))
                ++jend;
            chain_gamma(rank, ain.data(), perm.data(), aout.data(), b0.labels.data(), ki, ko, gamma);
            tuple_sign(b0.labels.data(), gamma);
            if (ki.size() != jend - i) throw Error(SYM_E_MISMATCH, "input blocks do not match the tree");
            for (int k = 0; k < rank; ++k) dims[k] = b0.shape[static_cast<size_t>(perm[static_cast<size_t>(k)])];
            std::vector<FmBlk> ins, outs;
            for (size_t k = i; k < jend; ++k) {
                if (key_of(in, in.blocks[k]) != ki[k - i]) throw Error(SYM_E_MISMATCH, "input blocks out of key order");
                ins.push_back(view(in.blocks[k], perm.data(), rank));
                ins.back().off += in_base;
            }
            int32_t olab[SYM_MAX_RANK];
            for (int l = 0; l < rank; ++l) olab[l] = b0.labels[static_cast<size_t>(perm[static_cast<size_t>(l)])];
            static const int32_t ident[kMaxRecoupleRank] = {0, 1, 2, 3, 4, 5, 6, 7};
            for (const auto& k : ko) {
                const int32_t oi = find_keyed(out, olab, k);
                if (oi < 0) throw Error(SYM_E_MISMATCH, "recoupled block missing from the output");
                outs.push_back(view(out.blocks[static_cast<size_t>(oi)], ident, rank));
                outs.back().off += out_base;
            }
            add_group(rank, dims, ins, outs, gamma);
            i = jend;
        }
        if (tiled_unfit) tiled = false;
        return;
    }
    if (rank != 4) throw Error(SYM_E_UNSUPPORTED, "rank-4 trees only");
    const TreeMoves mv = tree_moves(in.tree, perm.data(), out.tree);
    size_t i = 0;
    std::vector<int32_t> es, fs;
    std::vector<double> gamma;
    static const int32_t ident4[4] = {0, 1, 2, 3};
    while (i < in.blocks.size()) {
        const Block& b0 = in.blocks[i];
        size_t j = i;
        // input blocks of one label tuple are adjacent in canonical order
        while (j < in.blocks.size() &&
               std::equal(in.blocks[j].labels.begin(), in.blocks[j].labels.begin() + 4, b0.labels.begin()))
            ++j;
        tree_gamma(mv, b0.labels.data(), es, fs, gamma);
        tuple_sign(b0.labels.data(), gamma);
        const int n = static_cast<int>(es.size());
        if (static_cast<size_t>(n) != j - i) throw Error(SYM_E_MISMATCH, "input blocks do not match the tree");
        // output axis k is input axis perm[k]
        for (int k = 0; k < 4; ++k) dims[k] = b0.shape[static_cast<size_t>(perm[static_cast<size_t>(k)])];
        std::vector<FmBlk> ins, outs;
        for (size_t k = i; k < j; ++k) {
            if (in.blocks[k].internal != es[k - i]) throw Error(SYM_E_MISMATCH, "input intermediate spins out of order");
            ins.push_back(view(in.blocks[k], perm.data(), 4));
            ins.back().off += in_base;
        }
        int32_t olab[4];
        for (int l = 0; l < 4; ++l) olab[l] = b0.labels[static_cast<size_t>(perm[static_cast<size_t>(l)])];
        for (int32_t f : fs) {
            const int32_t oi = out.find_block(olab, f);
            if (oi < 0) throw Error(SYM_E_MISMATCH, "recoupled block missing from the output");
            outs.push_back(view(out.blocks[static_cast<size_t>(oi)], ident4, 4));
            outs.back().off += out_base;
        }
        add_group(4, dims, ins, outs, gamma);
        i = j;
    }
    if (tiled_unfit) tiled = false;
}

FusedLeg fuse_legs(const Leg& a, const Leg& b) {
    FusedLeg f;
    std::map<int32_t, int64_t> deg;
    for (size_t ia = 0; ia < a.label.size(); ++ia)
        for (size_t ib = 0; ib < b.label.size(); ++ib) {
            const int32_t ja = a.label[ia], jb = b.label[ib];
            for (int32_t c = ja > jb ? ja - jb : jb - ja; c <= ja + jb; c += 2) {
                f.offset[{ja, jb, c}] = deg[c];
                deg[c] += a.deg[ia] * b.deg[ib];
            }
        }
    for (const auto& kv : deg) {
        f.leg.label.push_back(kv.first);
        f.leg.deg.push_back(kv.second);
    }
    f.leg.arrow = a.arrow;
    return f;
}

void RecoupleProgram::build_fuse(const Desc& unf, const Desc& fus, int leg, bool to_fused) {
    if (unf.tree != SYM_TREE_CHAIN && unf.tree != SYM_TREE_OPERATOR && unf.tree != SYM_TREE_LEFT)
        throw Error(SYM_E_UNSUPPORTED, "FUSE and SPLIT take CHAIN, OPERATOR or LEFT tensors");
    src_dtype = to_fused ? unf.dtype : fus.dtype;
    dst_dtype = to_fused ? fus.dtype : unf.dtype;
    if (!recouple_dtypes_supported(src_dtype, dst_dtype))
        throw Error(SYM_E_DTYPE, "recoupling takes F32 -> F32, F32 -> BF16 or BF16 -> BF16");
    const int rank = unf.rank;
    const Leg& la = unf.legs[static_cast<size_t>(leg)];
    const Leg& lb = unf.legs[static_cast<size_t>(leg + 1)];
    const FusedLeg fl = fuse_legs(la, lb);
    const int side = la.arrow;
    int p = 0;   // position of the first fused leg in its chain
    for (int l = 0; l < leg; ++l) p += unf.legs[static_cast<size_t>(l)].arrow == side;
    std::vector<int32_t> arrows;
    for (const Leg& l : unf.legs) arrows.push_back(l.arrow);
    tiled = false;
    // views of the unfused shape inside a fused block: the fused axis as two
    // axes (t_a, t_b) at the offset of the pair
    auto fused_view = [&](const Block& fb, int64_t pair_off, const int64_t* dims) {
        FmBlk v{};
        const int64_t sf = fb.stride[static_cast<size_t>(leg)];
        v.off = fb.offset + pair_off * sf;
        int64_t span = 0;
        for (int k = 0; k < rank; ++k) {
            int64_t st;
            if (k < leg) st = fb.stride[static_cast<size_t>(k)];
            else if (k == leg) st = sf * dims[leg + 1];
            else if (k == leg + 1) st = sf;
            else st = fb.stride[static_cast<size_t>(k - 1)];
            if (st < 0 || st >= (int64_t{1} << 31)) throw Error(SYM_E_UNSUPPORTED, "block stride beyond 32 bits");
            span += (dims[k] - 1) * st;
            v.stride[k] = static_cast<int32_t>(st);
        }
        if (span >= (int64_t{1} << 31)) throw Error(SYM_E_UNSUPPORTED, "block span beyond 32 bits");
        return v;
    };
    static const int32_t ident[kMaxRecoupleRank] = {0, 1, 2, 3, 4, 5, 6, 7};
    size_t i = 0;
    while (i < unf.blocks.size()) {
        const Block& b0 = unf.blocks[i];
        size_t jend = i;
        while (jend < unf.blocks.size() &&
               std::equal(unf.blocks[jend].labels.begin(), unf.blocks[jend].labels.begin() + rank, b0.labels.begin()))
            ++jend;
        const std::vector<ChainBlock> cbs = chain_blocks(arrows, b0.labels.data(), rank);
        if (cbs.size() != jend - i) throw Error(SYM_E_MISMATCH, "blocks do not match the tree");
        const int32_t ja = b0.labels[static_cast<size_t>(leg)], jb = b0.labels[static_cast<size_t>(leg + 1)];
        int64_t dims[kMaxRecoupleRank];
        for (int k = 0; k < rank; ++k) dims[k] = b0.shape[static_cast<size_t>(k)];
        // fused labels: the pair replaced by the fused spin
        auto fused_labels = [&](int32_t c, int32_t* out) {
            int o = 0;
            for (int k = 0; k < rank; ++k) {
                if (k == leg + 1) continue;
                out[o++] = k == leg ? c : b0.labels[static_cast<size_t>(k)];
            }
        };
        // groups: blocks of this label tuple that agree on everything but s[p]
        std::map<std::pair<Seq, Seq>, std::vector<size_t>> groups;
        for (size_t k = 0; k < cbs.size(); ++k) {
            Seq a = cbs[k].a, b = cbs[k].b;
            Seq& sq = side == SYM_IN ? a : b;
            if (p >= 1) sq.erase(sq.begin() + p);   // p = 0: each block alone (its fused spin is s[1])
            groups[{a, b}].push_back(k);
        }
        for (const auto& kv : groups) {
            std::vector<FmBlk> ub, fbv;
            std::vector<double> g;
            const std::vector<size_t>& members = kv.second;
            const size_t n = members.size();
            std::vector<int32_t> fspins;
            if (p == 0) {
                const ChainBlock& cb = cbs[members[0]];
                fspins.push_back((side == SYM_IN ? cb.a : cb.b)[1]);
                g.assign(1, 1.0);
            } else {
                const ChainBlock& cb = cbs[members[0]];
                const Seq& sq = side == SYM_IN ? cb.a : cb.b;
                const int A = sq[static_cast<size_t>(p - 1)], J = sq[static_cast<size_t>(p + 1)];
                for (int32_t f = ja > jb ? ja - jb : jb - ja; f <= ja + jb; f += 2)
                    if (triangle(A, f, J)) fspins.push_back(f);
                if (fspins.size() != n) throw Error(SYM_E_MISMATCH, "fusion changes the multiplicity");
                g.assign(n * n, 0.0);
                for (size_t r = 0; r < n; ++r)
                    for (size_t c = 0; c < n; ++c) {
                        const Seq& sc = side == SYM_IN ? cbs[members[c]].a : cbs[members[c]].b;
                        const double v = fmove_coeff(A, ja, jb, J, sc[static_cast<size_t>(p)], fspins[r]);
                        // fuse: rows are fused spins; split: rows are the unfused blocks
                        if (to_fused) g[r * n + c] = v;
                        else g[c * n + r] = v;
                    }
            }
            for (size_t r = 0; r < n; ++r) {
                const Block& ublk = unf.blocks[i + members[r]];
                if (key_of(unf, ublk) != cbs[members[r]].key) throw Error(SYM_E_MISMATCH, "blocks out of key order");
                ub.push_back(view(ublk, ident, rank));
                // the fused block: fused labels, its chain with s[p] dropped (p >= 1) or s[0] = c (p = 0)
                const ChainBlock& cb = cbs[members[r]];
                Seq a = cb.a, b = cb.b;
                Seq& sq = side == SYM_IN ? a : b;
                const int32_t c = fspins[r];
                // the fused chain: s[p] dropped (p >= 1), or s[0] dropped so that
                // the fused spin s[1] = c leads (p = 0)
                sq.erase(sq.begin() + p);
                int32_t flab[SYM_MAX_RANK];
                fused_labels(c, flab);
                const std::vector<int32_t> key = chain_key(a, b);
                const int32_t fi = fus.tree == SYM_TREE_CHAIN
                                       ? fus.find_block_inner(flab, key.data(), static_cast<int32_t>(key.size()))
                                       : -1;
                if (fi < 0) throw Error(SYM_E_MISMATCH, "fused block missing");
                fbv.push_back(fused_view(fus.blocks[static_cast<size_t>(fi)], fl.offset.at({ja, jb, c}), dims));
            }
            if (to_fused) add_group(rank, dims, ub, fbv, g);
            else add_group(rank, dims, fbv, ub, g);
        }
        i = jend;
    }
}

namespace {

// One workgroup per task, dispatched in order, workgroup w on XCD w % 8:
// inside each window of g tasks (about the workgroups resident at once),
// XCD x takes a contiguous run of g / 8 tasks, so that neighbouring tasks,
// which share the cache lines at their edges, meet in one L2.  Measured on
// config 5: the tiled kernel's full reversal 0.973 against 1.00 ms; the
// element-wise kernel's tasks (16384 consecutive output entries each, few
// shared lines) ran 2 to 3 % slower that way and keep their order.
template <typename Task>
void xcd_runs(std::vector<Task>& v, size_t begin, size_t end) {
    constexpr int64_t g = 2048, per = g / 8;
    std::vector<Task> seq(v.begin() + static_cast<std::ptrdiff_t>(begin), v.begin() + static_cast<std::ptrdiff_t>(end));
    const int64_t n = static_cast<int64_t>(seq.size());
    for (int64_t r0 = 0; r0 + g <= n; r0 += g)
        for (int64_t w = 0; w < g; ++w)
            v[begin + static_cast<size_t>(r0 + w)] = seq[static_cast<size_t>(r0 + (w % 8) * per + w / 8)];
}

}  // namespace

void RecoupleProgram::upload(const Allocator& alloc, Deferred* deferred) {
    // the tasks of small tuples first: they run in the high-occupancy kernel
    auto small = [&](const FmTask& t) { return groups[static_cast<size_t>(t.group)].n <= kRecoupleSmallN; };
    n_small = static_cast<int32_t>(std::stable_partition(tasks.begin(), tasks.end(), small) - tasks.begin());
    auto tsmall = [&](const FtTask& t) { return tgroups[static_cast<size_t>(t.group)].n <= kRecoupleTiledSmallN; };
    n_tsmall = static_cast<int32_t>(std::stable_partition(ttasks.begin(), ttasks.end(), tsmall) - ttasks.begin());
    xcd_runs(ttasks, 0, static_cast<size_t>(n_tsmall));
    xcd_runs(ttasks, static_cast<size_t>(n_tsmall), ttasks.size());
    d_groups = upload_vec(alloc, groups, deferred);
    d_in = upload_vec(alloc, in_blks, deferred);
    d_out = upload_vec(alloc, out_blks, deferred);
    d_coef = upload_vec(alloc, coef, deferred);
    d_tasks = upload_vec(alloc, tasks, deferred);
    d_tgroups = upload_vec(alloc, tgroups, deferred);
    d_ttasks = upload_vec(alloc, ttasks, deferred);
}

hipError_t RecoupleProgram::launch(const PtrTable& bufs, int in_buf, int out_buf, hipStream_t s) const {
    if (tasks.empty()) return hipSuccess;
    if (tiled)
        return launch_recouple_tiled(src_dtype, dst_dtype, static_cast<const FtGroup*>(d_tgroups->ptr),
                                     static_cast<const FmBlk*>(d_in->ptr),
                                     static_cast<const FmBlk*>(d_out->ptr), static_cast<const double*>(d_coef->ptr),
                                     static_cast<const FtTask*>(d_ttasks->ptr), n_tsmall,
                                     static_cast<int32_t>(ttasks.size()), bufs, in_buf, out_buf, s);
    return launch_recouple(src_dtype, dst_dtype, static_cast<const FmGroup*>(d_groups->ptr),
                           static_cast<const FmBlk*>(d_in->ptr),
                           static_cast<const FmBlk*>(d_out->ptr), static_cast<const double*>(d_coef->ptr),
                           static_cast<const FmTask*>(d_tasks->ptr), n_small, static_cast<int32_t>(tasks.size()), bufs,
                           in_buf, out_buf, s);
}

}  // namespace sym
