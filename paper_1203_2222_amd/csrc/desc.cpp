// Tensor descriptors: validation, allowed-block enumeration and the
// sector-major layout (host side, pure integer work).
//
// U(1) rule (invariance condition eq:Tinv with exp(i r q) on every leg,
// conjugated on 'in' legs): a label tuple is allowed when
// sum(q, out) - sum(q, in) == qtot.  SU(2) rule: every node of the tree obeys
// the fusion rule eq:fusionrules.  Blocks are the degeneracy tensors of the
// canonical form (eq:datak).
#include <algorithm>
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

int32_t Desc::find_block(const int32_t* labels, int32_t internal) const {
    auto it = block_index.find(label_key(labels, rank, internal));
    return it == block_index.end() ? -1 : it->second;
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
    if (rank != 4) throw Error(SYM_E_UNSUPPORTED, "SU(2) tensors here have rank 4");
    if (qtot != 0) throw Error(SYM_E_ARG, "SU(2) tensors are invariant (qtot = 0)");
    static const int32_t op_arrows[4] = {SYM_IN, SYM_IN, SYM_OUT, SYM_OUT};
    static const int32_t fuse_arrows[4] = {SYM_IN, SYM_IN, SYM_IN, SYM_OUT};
    const int32_t* want = nullptr;
    if (tree == SYM_TREE_OPERATOR) want = op_arrows;
    else if (tree == SYM_TREE_LEFT || tree == SYM_TREE_RIGHT) want = fuse_arrows;
    else throw Error(SYM_E_ARG, "SU(2) tensors need the OPERATOR, LEFT or RIGHT tree");
    for (int i = 0; i < 4; ++i)
        if (legs[static_cast<size_t>(i)].arrow != want[i]) throw Error(SYM_E_ARROW, "arrows do not match the SU(2) tree");
    for (const Leg& l : legs)
        for (int32_t lab : l.label)
            if (lab < 0) throw Error(SYM_E_CHARGE, "SU(2) labels are 2j >= 0");
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
        b.labels = t.lab;
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
                b.labels = t.lab;
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
            b.labels = t.lab;
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
    if (group == SYM_SU2 && opts.trans && n_row != 2)
        throw Error(SYM_E_UNSUPPORTED, "transposed SU(2) layout needs n_row = 2");
    if (is_abelian(group)) build_u1(*d);
    else build_su2(*d);
    for (size_t i = 0; i < d->blocks.size(); ++i)
        d->block_index[label_key(d->blocks[i].labels.data(), d->rank, d->blocks[i].internal)] = static_cast<int32_t>(i);
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
