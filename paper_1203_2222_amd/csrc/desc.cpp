// Tensor descriptors: validation, allowed-block enumeration and the
// sector-major layout (host side, pure integer work).
//
// U(1) rule (invariance condition eq:Tinv with exp(i r q) on every leg,
// conjugated on 'in' legs): a label tuple is allowed when
// sum(q, out) - sum(q, in) == qtot.  SU(2) rule: every node of the tree obeys
// the fusion rule eq:fusionrules.  Blocks are the degeneracy tensors of the
// canonical form (eq:datak).
#include <algorithm>
#include <map>
#include <set>
#include <sstream>

#include "internal.hpp"

namespace sym {

size_t dtype_size(int32_t dt) { return dt == SYM_BF16 ? 2 : 4; }

std::string label_key(const int32_t* labels, int n, int32_t internal) {
    std::string s(static_cast<size_t>(n + 1) * sizeof(int32_t), '\0');
    if (n) std::memcpy(&s[0], labels, static_cast<size_t>(n) * sizeof(int32_t));
    std::memcpy(&s[static_cast<size_t>(n) * sizeof(int32_t)], &internal, sizeof(int32_t));
    return s;
}

std::string inner_key(const int32_t* labels, int n, const int32_t* inner, int n_inner) {
    std::string s(static_cast<size_t>(n + n_inner + 1) * sizeof(int32_t), '\0');
    if (n) std::memcpy(&s[0], labels, static_cast<size_t>(n) * sizeof(int32_t));
    if (n_inner) std::memcpy(&s[static_cast<size_t>(n) * sizeof(int32_t)], inner, static_cast<size_t>(n_inner) * sizeof(int32_t));
    const int32_t tag = -2 - n_inner;   // distinct from any rank-4 internal spin
    std::memcpy(&s[static_cast<size_t>(n + n_inner) * sizeof(int32_t)], &tag, sizeof(int32_t));
    return s;
}

int32_t Desc::find_block(const int32_t* labels, int32_t internal) const {
    auto it = block_index.find(label_key(labels, rank, internal));
    return it == block_index.end() ? -1 : it->second;
}

int32_t Desc::find_block_inner(const int32_t* labels, const int32_t* inner, int32_t n_inner) const {
    auto it = block_index.find(inner_key(labels, rank, inner, n_inner));
    return it == block_index.end() ? -1 : it->second;
}

int32_t Desc::find_block(const int32_t* labels, const Block& like) const {
    if (tree == SYM_TREE_CHAIN) return find_block_inner(labels, like.inner.data(), like.n_inner);
    return find_block(labels, like.internal);
}

std::vector<Seq> chain_sequences(const std::vector<int32_t>& spins) {
    std::vector<Seq> out;
    if (spins.empty()) {
        out.emplace_back();
        return out;
    }
    out.push_back(Seq{spins[0]});
    for (size_t k = 1; k < spins.size(); ++k) {
        std::vector<Seq> next;
        for (const Seq& q : out) {
            const int32_t a = q.back(), j = spins[k];
            for (int32_t c = a > j ? a - j : j - a; c <= a + j; c += 2) {
                Seq r = q;
                r.push_back(c);
                next.push_back(std::move(r));
            }
        }
        out.swap(next);
    }
    return out;
}

std::vector<int32_t> chain_key(const Seq& a, const Seq& b) {
    const size_t n = a.size(), m = b.size();
    std::vector<int32_t> k;
    for (size_t i = 1; i + 1 < n; ++i) k.push_back(a[i]);
    if (n >= 2 && m >= 2) k.push_back(a.back());
    for (size_t i = 1; i + 1 < m; ++i) k.push_back(b[i]);
    return k;
}

std::vector<ChainBlock> chain_blocks(const std::vector<int32_t>& arrows, const int32_t* labels, int rank) {
    std::vector<int32_t> sin, sout;
    for (int l = 0; l < rank; ++l) (arrows[static_cast<size_t>(l)] == SYM_IN ? sin : sout).push_back(labels[l]);
    const std::vector<Seq> A = chain_sequences(sin), B = chain_sequences(sout);
    std::vector<ChainBlock> out;
    for (const Seq& a : A)
        for (const Seq& b : B)
            if (chain_total(a) == chain_total(b)) out.push_back(ChainBlock{a, b, chain_key(a, b)});
    std::sort(out.begin(), out.end(), [](const ChainBlock& x, const ChainBlock& y) { return x.key < y.key; });
    return out;
}

int32_t Desc::find_sector(int32_t label) const {
    for (size_t i = 0; i < sectors.size(); ++i)
        if (sectors[i].label == label) return static_cast<int32_t>(i);
    return -1;
}

std::vector<Leg> permute_legs(const std::vector<Leg>& legs, const std::vector<int32_t>& perm) {
    std::vector<Leg> out;
    out.reserve(perm.size());
    for (int32_t p : perm) out.push_back(legs[static_cast<size_t>(p)]);
    return out;
}

namespace {

int64_t round_up(int64_t x, int64_t a) { return a <= 1 ? x : (x + a - 1) / a * a; }

// All label tuples over legs [first, first+count), lexicographic.
std::vector<Tuple> enumerate(const std::vector<Leg>& legs, int first, int count) {
    std::vector<Tuple> out;
    std::vector<size_t> idx(static_cast<size_t>(count), 0);
    for (int i = 0; i < count; ++i)
        if (legs[static_cast<size_t>(first + i)].label.empty()) return out;
    while (true) {
        Tuple t;
        t.n = count;
        for (int i = 0; i < count; ++i) {
            const Leg& l = legs[static_cast<size_t>(first + i)];
            t.lab[static_cast<size_t>(i)] = l.label[idx[static_cast<size_t>(i)]];
            t.dim *= l.deg[idx[static_cast<size_t>(i)]];
        }
        out.push_back(t);
        int k = count - 1;
        while (k >= 0) {
            size_t& v = idx[static_cast<size_t>(k)];
            if (++v < legs[static_cast<size_t>(first + k)].label.size()) break;
            v = 0;
            --k;
        }
        if (k < 0) break;
    }
    return out;
}

int64_t deg_of(const Leg& l, int32_t label) {
    for (size_t i = 0; i < l.label.size(); ++i)
        if (l.label[i] == label) return l.deg[i];
    return 0;
}

void validate(int32_t group, const std::vector<Leg>& legs, int32_t n_row, int32_t tree, int32_t qtot,
              int32_t dtype) {
    const int rank = static_cast<int>(legs.size());
    if (!is_abelian(group) && group != SYM_SU2) throw Error(SYM_E_ARG, "unknown group");
    if (rank > SYM_MAX_RANK) throw Error(SYM_E_ARG, "rank exceeds SYM_MAX_RANK");
    if (n_row < 0 || n_row > rank) throw Error(SYM_E_ARG, "n_row outside [0, rank]");
    if (dtype != SYM_F32 && dtype != SYM_BF16) throw Error(SYM_E_DTYPE, "dtype must be F32 or BF16");
    for (const Leg& l : legs) {
        if (l.arrow != SYM_IN && l.arrow != SYM_OUT) throw Error(SYM_E_ARG, "arrow must be SYM_IN or SYM_OUT");
        if (l.label.size() != l.deg.size()) throw Error(SYM_E_ARG, "labels and degeneracies differ in count");
        for (size_t i = 0; i < l.label.size(); ++i) {
            if (l.deg[i] < 1) throw Error(SYM_E_ARG, "degeneracy must be >= 1");
            if (i && l.label[i] <= l.label[i - 1]) throw Error(SYM_E_CHARGE, "labels must be strictly ascending");
        }
    }
    if (is_abelian(group)) {
        if (tree != SYM_TREE_NONE) throw Error(SYM_E_ARG, "Abelian tensors take SYM_TREE_NONE");
        if (group == SYM_Z2 || group == SYM_Z2F) {
            if (qtot != 0 && qtot != 1) throw Error(SYM_E_CHARGE, "parity qtot must be 0 or 1");
            for (const Leg& l : legs)
                for (int32_t lab : l.label)
                    if (lab != 0 && lab != 1) throw Error(SYM_E_CHARGE, "parity labels are 0 or 1");
        } else if (group == SYM_U1U1) {
            auto ok = [](int32_t v) {
                const int32_t q1 = (v + 32768) >> 16, q2 = v - q1 * 65536;
                return q1 >= -2048 && q1 < 2048 && q2 >= -2048 && q2 < 2048;
            };
            if (!ok(qtot)) throw Error(SYM_E_CHARGE, "U(1) x U(1) qtot components outside [-2048, 2048)");
            for (const Leg& l : legs)
                for (int32_t lab : l.label)
                    if (!ok(lab)) throw Error(SYM_E_CHARGE, "U(1) x U(1) label components outside [-2048, 2048)");
        }
        return;
    }
    if (qtot != 0) throw Error(SYM_E_ARG, "SU(2) tensors are invariant (qtot = 0)");
    for (const Leg& l : legs)
        for (int32_t lab : l.label)
            if (lab < 0) throw Error(SYM_E_CHARGE, "SU(2) labels are 2j >= 0");
    if (tree == SYM_TREE_CHAIN) {
        if (rank < 1) throw Error(SYM_E_ARG, "CHAIN tensors have rank 1..SYM_MAX_RANK");
        // sector-major layouts: the first n_row legs are the first incoming
        // legs of the chain (rows), the sector their coupled spin
        if (n_row > 0 && n_row < rank)
            for (int i = 0; i < n_row; ++i)
                if (legs[static_cast<size_t>(i)].arrow != SYM_IN)
                    throw Error(SYM_E_UNSUPPORTED, "a CHAIN sector layout needs its row legs incoming");
        return;
    }
    if (rank != 4) throw Error(SYM_E_UNSUPPORTED, "OPERATOR, LEFT and RIGHT trees have rank 4 (use the CHAIN tree)");
    static const int32_t op_arrows[4] = {SYM_IN, SYM_IN, SYM_OUT, SYM_OUT};
    static const int32_t fuse_arrows[4] = {SYM_IN, SYM_IN, SYM_IN, SYM_OUT};
    const int32_t* want = nullptr;
    if (tree == SYM_TREE_OPERATOR) want = op_arrows;
    else if (tree == SYM_TREE_LEFT || tree == SYM_TREE_RIGHT) want = fuse_arrows;
    else throw Error(SYM_E_ARG, "SU(2) tensors need the OPERATOR, LEFT, RIGHT or CHAIN tree");
    for (int i = 0; i < 4; ++i)
        if (legs[static_cast<size_t>(i)].arrow != want[i]) throw Error(SYM_E_ARROW, "arrows do not match the SU(2) tree");
    if (!(n_row == 0 || n_row == 4 || n_row == 2)) throw Error(SYM_E_UNSUPPORTED, "SU(2) n_row must be 0, 2 or 4");
    if (n_row == 2 && tree == SYM_TREE_RIGHT)
        throw Error(SYM_E_UNSUPPORTED, "the RIGHT tree has no 2|2 sector layout");
}

// Intermediate spins of a rank-4 SU(2) label tuple on a tree.
std::vector<int32_t> su2_internals(int32_t tree, const int32_t* j) {
    std::vector<int32_t> out;
    const int32_t hi = 2 * std::max(std::max(j[0], j[1]), std::max(j[2], j[3])) + 1;
    for (int32_t e = 0; e <= hi; ++e) {
        bool ok = false;
        if (tree == SYM_TREE_OPERATOR) ok = triangle(j[0], j[1], e) && triangle(j[2], j[3], e);
        else if (tree == SYM_TREE_LEFT) ok = triangle(j[0], j[1], e) && triangle(e, j[2], j[3]);
        else if (tree == SYM_TREE_RIGHT) ok = triangle(j[1], j[2], e) && triangle(j[0], e, j[3]);
        if (ok) out.push_back(e);
    }
    return out;
}

// Fill offsets/strides of a block inside its sector matrix.
void place_block(Desc& d, Block& b, const Sector& s, int64_t row_off, int64_t col_off) {
    const bool tr = d.opts.trans;
    b.offset = s.offset + (tr ? col_off * s.ld + row_off : row_off * s.ld + col_off);
    int64_t acc = 1;
    for (int l = d.n_row - 1; l >= 0; --l) {
        b.stride[static_cast<size_t>(l)] = acc * (tr ? 1 : s.ld);
        acc *= b.shape[static_cast<size_t>(l)];
    }
    acc = 1;
    for (int l = d.rank - 1; l >= d.n_row; --l) {
        b.stride[static_cast<size_t>(l)] = acc * (tr ? s.ld : 1);
        acc *= b.shape[static_cast<size_t>(l)];
    }
}

void finish_sectors(Desc& d) {
    int64_t off = 0;
    for (Sector& s : d.sectors) {
        s.rows = 0;
        for (const Tuple& t : s.row_tuples) { s.row_off.push_back(s.rows); s.rows += t.dim; }
        s.cols = 0;
        for (const Tuple& t : s.col_tuples) { s.col_off.push_back(s.cols); s.cols += t.dim; }
        s.ld = round_up(d.opts.trans ? s.rows : s.cols, d.opts.ld_align);
        // BF16 GEMM operand layouts: a row pitch of 32 KB or more that is a
        // multiple of 16 KB gets one more cache line.  Measured on single
        // square sectors with the grouped BF16 GEMM: 16384, 24576 and 32768
        // columns (32, 48, 64 KB rows) ran 17, 11 and 19 % faster padded,
        // 8192 (16 KB) 6 % slower, the other pitches tried unchanged.
        if (d.opts.ld_align > 1 && d.dtype == SYM_BF16) {
            const int64_t row_bytes = s.ld * static_cast<int64_t>(dtype_size(d.dtype));
            if (row_bytes >= 32768 && row_bytes % 16384 == 0) s.ld += d.opts.ld_align;
        }
        off = round_up(off, d.opts.base_align);
        s.offset = off;
        off += (d.opts.trans ? s.cols : s.rows) * s.ld;
    }
    d.numel = off;
}

// Abelian groups: the sector of a row tuple is the charge flowing in through
// the row legs (folded for the parity groups); a column tuple joins the
// sector whose charge it carries out (minus qtot).  With the encoded
// U(1) x U(1) labels, bounded components make the sum of codes the code of
// the componentwise sums, so equality of codes is the componentwise rule.
void build_u1(Desc& d) {
    const int rank = d.rank, nr = d.n_row;
    std::vector<Tuple> rows = enumerate(d.legs, 0, nr);
    std::vector<Tuple> cols = enumerate(d.legs, nr, rank - nr);
    auto rho = [&](const Tuple& t) {
        int32_t s = 0;
        for (int i = 0; i < t.n; ++i) s += (d.legs[static_cast<size_t>(i)].arrow == SYM_IN ? 1 : -1) * t.lab[static_cast<size_t>(i)];
        return fold(d.group, s);
    };
    auto kap = [&](const Tuple& t) {
        int32_t s = 0;
        for (int i = 0; i < t.n; ++i) s += (d.legs[static_cast<size_t>(nr + i)].arrow == SYM_OUT ? 1 : -1) * t.lab[static_cast<size_t>(i)];
        return fold(d.group, s - d.qtot);
    };
    std::map<int32_t, std::vector<Tuple>> rmap, cmap;
    for (const Tuple& t : rows) rmap[rho(t)].push_back(t);
    for (const Tuple& t : cols) cmap[kap(t)].push_back(t);
    for (auto& kv : rmap) {
        auto it = cmap.find(kv.first);
        if (it == cmap.end()) continue;
        Sector s;
        s.label = kv.first;
        s.row_tuples = kv.second;
        s.col_tuples = it->second;
        d.sectors.push_back(std::move(s));
    }
    finish_sectors(d);
    // tuple -> (sector, offset) lookups
    std::unordered_map<std::string, std::pair<int32_t, int64_t>> rpos, cpos;
    for (size_t si = 0; si < d.sectors.size(); ++si) {
        const Sector& s = d.sectors[si];
        for (size_t i = 0; i < s.row_tuples.size(); ++i)
            rpos[label_key(s.row_tuples[i].lab.data(), nr, 0)] = {static_cast<int32_t>(si), s.row_off[i]};
        for (size_t i = 0; i < s.col_tuples.size(); ++i)
            cpos[label_key(s.col_tuples[i].lab.data(), rank - nr, 0)] = {static_cast<int32_t>(si), s.col_off[i]};
    }
    std::vector<Tuple> all = enumerate(d.legs, 0, rank);
    for (const Tuple& t : all) {
        auto r = rpos.find(label_key(t.lab.data(), nr, 0));
        auto c = cpos.find(label_key(t.lab.data() + nr, rank - nr, 0));
        if (r == rpos.end() || c == cpos.end() || r->second.first != c->second.first) continue;
        Block b;
        std::copy(t.lab.begin(), t.lab.begin() + SYM_MAX_RANK, b.labels.begin());
        b.internal = -1;
        for (int i = 0; i < rank; ++i) b.shape[static_cast<size_t>(i)] = deg_of(d.legs[static_cast<size_t>(i)], t.lab[static_cast<size_t>(i)]);
        b.size = t.dim;
        b.sector = r->second.first;
        place_block(d, b, d.sectors[static_cast<size_t>(b.sector)], r->second.second, c->second.second);
        d.blocks.push_back(b);
    }
}

void build_su2(Desc& d) {
    std::vector<Tuple> all = enumerate(d.legs, 0, 4);
    if (d.n_row == 2) {
        std::vector<Tuple> pairs_r = enumerate(d.legs, 0, 2);
        std::vector<Tuple> pairs_c = enumerate(d.legs, 2, 2);
        std::map<int32_t, std::vector<Tuple>> rmap, cmap;
        const int32_t emax = 64;
        for (const Tuple& t : pairs_r)
            for (int32_t e = 0; e <= emax; ++e)
                if (triangle(t.lab[0], t.lab[1], e)) rmap[e].push_back(t);
        for (const Tuple& t : pairs_c)
            for (int32_t e = 0; e <= emax; ++e) {
                bool ok = d.tree == SYM_TREE_OPERATOR ? triangle(t.lab[0], t.lab[1], e) : triangle(e, t.lab[0], t.lab[1]);
                if (ok) cmap[e].push_back(t);
            }
        for (auto& kv : rmap) {
            auto it = cmap.find(kv.first);
            if (it == cmap.end()) continue;
            Sector s;
            s.label = kv.first;
            s.row_tuples = kv.second;
            s.col_tuples = it->second;
            d.sectors.push_back(std::move(s));
        }
        finish_sectors(d);
        std::unordered_map<std::string, int64_t> rpos, cpos;
        for (const Sector& s : d.sectors) {
            for (size_t i = 0; i < s.row_tuples.size(); ++i)
                rpos[label_key(s.row_tuples[i].lab.data(), 2, s.label)] = s.row_off[i];
            for (size_t i = 0; i < s.col_tuples.size(); ++i)
                cpos[label_key(s.col_tuples[i].lab.data(), 2, s.label)] = s.col_off[i];
        }
        for (const Tuple& t : all) {
            for (int32_t e : su2_internals(d.tree, t.lab.data())) {
                Block b;
                std::copy(t.lab.begin(), t.lab.begin() + SYM_MAX_RANK, b.labels.begin());
                b.internal = e;
                for (int i = 0; i < 4; ++i) b.shape[static_cast<size_t>(i)] = deg_of(d.legs[static_cast<size_t>(i)], t.lab[static_cast<size_t>(i)]);
                b.size = t.dim;
                b.sector = d.find_sector(e);
                const Sector& s = d.sectors[static_cast<size_t>(b.sector)];
                place_block(d, b, s, rpos.at(label_key(t.lab.data(), 2, e)), cpos.at(label_key(t.lab.data() + 2, 2, e)));
                d.blocks.push_back(b);
            }
        }
        return;
    }
    // canonical block list: one sector holding every block back to back
    Sector s;
    s.label = 0;
    d.sectors.push_back(s);
    int64_t off = 0;
    for (const Tuple& t : all) {
        for (int32_t e : su2_internals(d.tree, t.lab.data())) {
            Block b;
            std::copy(t.lab.begin(), t.lab.begin() + SYM_MAX_RANK, b.labels.begin());
            b.internal = e;
            for (int i = 0; i < 4; ++i) b.shape[static_cast<size_t>(i)] = deg_of(d.legs[static_cast<size_t>(i)], t.lab[static_cast<size_t>(i)]);
            b.size = t.dim;
            b.sector = 0;
            b.offset = off;
            int64_t acc = 1;
            for (int l = 3; l >= 0; --l) { b.stride[static_cast<size_t>(l)] = acc; acc *= b.shape[static_cast<size_t>(l)]; }
            off += b.size;
            d.blocks.push_back(b);
        }
    }
    Sector& s0 = d.sectors[0];
    if (d.n_row == 4) { s0.rows = off; s0.cols = 1; s0.ld = 1; }
    else { s0.rows = 1; s0.cols = off; s0.ld = off; }
    d.numel = off;
}

// CHAIN tree (any rank).  Canonical block list for n_row = 0 or rank;
// otherwise sector-major for the bipartition after the first n_row
// (incoming) legs: the sector of a block is the coupled spin a_{n_row-1} of
// its row legs, a row tuple is (row labels, a_1 .. a_{n_row-2}) and a column
// tuple the remaining labels with the remaining intermediate spins
// (a_{n_row} .. a_{n-1}, b_1 .. b_{m-2}).  Row and column tuples are
// ordered lexicographically, labels first.
void build_chain(Desc& d) {
    const int rank = d.rank, k = d.n_row;
    std::vector<int32_t> arrows;
    int n_in = 0;
    for (const Leg& l : d.legs) {
        arrows.push_back(l.arrow);
        n_in += l.arrow == SYM_IN;
    }
    std::vector<Tuple> all = enumerate(d.legs, 0, rank);
    auto shape_of = [&](Block& b, const Tuple& t) {
        for (int i = 0; i < rank; ++i) b.shape[static_cast<size_t>(i)] = deg_of(d.legs[static_cast<size_t>(i)], t.lab[static_cast<size_t>(i)]);
        b.size = t.dim;
    };
    auto set_key = [](Block& b, const std::vector<int32_t>& key) {
        if (key.size() > static_cast<size_t>(SYM_MAX_RANK)) throw Error(SYM_E_UNSUPPORTED, "too many intermediate spins");
        b.n_inner = static_cast<int32_t>(key.size());
        for (size_t i = 0; i < key.size(); ++i) b.inner[i] = key[i];
    };
    if (k == 0 || k == rank) {
        Sector s;
        s.label = 0;
        d.sectors.push_back(s);
        int64_t off = 0;
        for (const Tuple& t : all) {
            for (const ChainBlock& cb : chain_blocks(arrows, t.lab.data(), rank)) {
                Block b;
                b.labels = {};
                for (int i = 0; i < rank; ++i) b.labels[static_cast<size_t>(i)] = t.lab[static_cast<size_t>(i)];
                set_key(b, cb.key);
                shape_of(b, t);
                b.sector = 0;
                b.offset = off;
                int64_t acc = 1;
                for (int l = rank - 1; l >= 0; --l) { b.stride[static_cast<size_t>(l)] = acc; acc *= b.shape[static_cast<size_t>(l)]; }
                off += b.size;
                d.blocks.push_back(b);
            }
        }
        Sector& s0 = d.sectors[0];
        if (k == rank) { s0.rows = off; s0.cols = 1; s0.ld = 1; }
        else { s0.rows = 1; s0.cols = off; s0.ld = off; }
        d.numel = off;
        return;
    }
    // row / column tuples of every block, grouped by sector
    struct Item { Tuple t; Tuple row, col; int32_t sector; ChainBlock cb; };
    std::vector<Item> items;
    std::map<int32_t, std::set<std::vector<int32_t>>> rset, cset;
    std::map<std::vector<int32_t>, Tuple> tuple_of;
    auto make_tuple = [&](const int32_t* labs, int nl, int first_leg, const std::vector<int32_t>& ints) {
        Tuple u;
        u.n = nl + static_cast<int32_t>(ints.size());
        if (u.n > 2 * SYM_MAX_RANK) throw Error(SYM_E_UNSUPPORTED, "tuple too long");
        for (int i = 0; i < nl; ++i) {
            u.lab[static_cast<size_t>(i)] = labs[i];
            u.dim *= deg_of(d.legs[static_cast<size_t>(first_leg + i)], labs[i]);
        }
        for (size_t i = 0; i < ints.size(); ++i) u.lab[static_cast<size_t>(nl) + i] = ints[i];
        return u;
    };
    auto vec_of = [](const Tuple& u) { return std::vector<int32_t>(u.lab.begin(), u.lab.begin() + u.n); };
    for (const Tuple& t : all) {
        for (const ChainBlock& cb : chain_blocks(arrows, t.lab.data(), rank)) {
            // the first k legs are the first k incoming ones: a_0 .. a_{k-1}
            std::vector<int32_t> rint(cb.a.begin() + 1, cb.a.begin() + (k >= 2 ? k - 1 : 1));
            if (k < 2) rint.clear();
            std::vector<int32_t> cint(cb.a.begin() + k, cb.a.end());
            for (size_t i = 1; i + 1 < cb.b.size(); ++i) cint.push_back(cb.b[i]);
            Item it{t, make_tuple(t.lab.data(), k, 0, rint), make_tuple(t.lab.data() + k, rank - k, k, cint),
                    cb.a[static_cast<size_t>(k - 1)], cb};
            rset[it.sector].insert(vec_of(it.row));
            cset[it.sector].insert(vec_of(it.col));
            tuple_of[vec_of(it.row)] = it.row;
            items.push_back(std::move(it));
        }
    }
    std::map<std::pair<int32_t, std::vector<int32_t>>, Tuple> ctuple;
    for (const Item& it : items) ctuple[{it.sector, vec_of(it.col)}] = it.col;
    for (auto& kv : rset) {
        Sector s;
        s.label = kv.first;
        for (const auto& v : kv.second) s.row_tuples.push_back(tuple_of.at(v));
        for (const auto& v : cset.at(kv.first)) s.col_tuples.push_back(ctuple.at({kv.first, v}));
        d.sectors.push_back(std::move(s));
    }
    finish_sectors(d);
    std::map<std::pair<int32_t, std::vector<int32_t>>, int64_t> rpos, cpos;
    for (const Sector& s : d.sectors) {
        for (size_t i = 0; i < s.row_tuples.size(); ++i) rpos[{s.label, vec_of(s.row_tuples[i])}] = s.row_off[i];
        for (size_t i = 0; i < s.col_tuples.size(); ++i) cpos[{s.label, vec_of(s.col_tuples[i])}] = s.col_off[i];
    }
    for (const Item& it : items) {
        Block b;
        for (int i = 0; i < rank; ++i) b.labels[static_cast<size_t>(i)] = it.t.lab[static_cast<size_t>(i)];
        set_key(b, it.cb.key);
        shape_of(b, it.t);
        b.sector = d.find_sector(it.sector);
        place_block(d, b, d.sectors[static_cast<size_t>(b.sector)], rpos.at({it.sector, vec_of(it.row)}),
                    cpos.at({it.sector, vec_of(it.col)}));
        d.blocks.push_back(b);
    }
    (void)n_in;
}

}  // namespace

DescPtr make_desc(int32_t group, const std::vector<Leg>& legs, int32_t n_row, int32_t tree, int32_t qtot,
                  int32_t dtype, const LayoutOpts& opts) {
    validate(group, legs, n_row, tree, qtot, dtype);
    auto d = std::make_shared<Desc>();
    d->group = group;
    d->rank = static_cast<int32_t>(legs.size());
    d->n_row = n_row;
    d->tree = tree;
    d->qtot = qtot;
    d->dtype = dtype;
    d->opts = opts;
    d->legs = legs;
    if (group == SYM_SU2 && tree != SYM_TREE_CHAIN && opts.trans && n_row != 2)
        throw Error(SYM_E_UNSUPPORTED, "transposed SU(2) layout needs n_row = 2");
    if (group == SYM_SU2 && tree == SYM_TREE_CHAIN && opts.trans && (n_row == 0 || n_row == d->rank))
        throw Error(SYM_E_UNSUPPORTED, "transposed CHAIN layout needs a sector bipartition");
    if (is_abelian(group)) build_u1(*d);
    else if (tree == SYM_TREE_CHAIN) build_chain(*d);
    else build_su2(*d);
    for (size_t i = 0; i < d->blocks.size(); ++i) {
        const Block& b = d->blocks[i];
        d->block_index[tree == SYM_TREE_CHAIN ? inner_key(b.labels.data(), d->rank, b.inner.data(), b.n_inner)
                                              : label_key(b.labels.data(), d->rank, b.internal)] = static_cast<int32_t>(i);
    }
    std::ostringstream k;
    k << group << '|' << d->rank << '|' << n_row << '|' << tree << '|' << qtot << '|' << dtype << '|'
      << opts.trans << '|' << opts.ld_align << '|' << opts.base_align;
    for (const Leg& l : legs) {
        k << "|" << l.arrow << ':';
        for (size_t i = 0; i < l.label.size(); ++i) k << l.label[i] << 'x' << l.deg[i] << ',';
    }
    d->key = k.str();
    return d;
}

}  // namespace sym
