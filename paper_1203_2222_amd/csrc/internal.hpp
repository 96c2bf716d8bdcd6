// Internal declarations of the symtensor library (host side).
#pragma once

#include <array>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "symtensor.h"

namespace sym {

// Error carried to the C-ABI boundary, where it becomes a status code.
struct Error : std::runtime_error {
    int32_t status;
    Error(int32_t s, const std::string& m) : std::runtime_error(m), status(s) {}
};

// Abelian groups: one int32 label per irrep, fusion by (signed) addition
// followed by fold() (identity for U(1) and the encoded U(1) x U(1), modulo 2
// for the parity groups).
inline bool is_abelian(int32_t g) { return g == SYM_U1 || g == SYM_Z2 || g == SYM_U1U1 || g == SYM_Z2F; }
inline int32_t fold(int32_t g, int32_t s) { return (g == SYM_Z2 || g == SYM_Z2F) ? ((s % 2) + 2) % 2 : s; }
inline int32_t combine_qtot(int32_t g, int32_t a, int32_t b) { return fold(g, a + b); }

struct Leg {
    std::vector<int32_t> label;
    std::vector<int64_t> deg;
    int32_t arrow = SYM_IN;
    bool operator==(const Leg& o) const {
        return label == o.label && deg == o.deg && arrow == o.arrow;
    }
    bool same_spectrum(const Leg& o) const { return label == o.label && deg == o.deg; }
};

// A tuple of labels on a subset of legs (for SU(2) CHAIN trees followed by
// the intermediate spins that belong to that side), with its degeneracy
// product.
struct Tuple {
    std::array<int32_t, 2 * SYM_MAX_RANK> lab{};
    int32_t n = 0;
    int64_t dim = 1;
    bool operator==(const Tuple& o) const {
        if (n != o.n) return false;
        for (int i = 0; i < n; ++i)
            if (lab[i] != o.lab[i]) return false;
        return true;
    }
};

struct Block {
    std::array<int32_t, SYM_MAX_RANK> labels{};
    int32_t internal = -1;   // SU(2) intermediate spin (doubled) of a rank-4 tree; -1 otherwise
    // SU(2) CHAIN tree: the block's free intermediate spins (see chain_key)
    std::array<int32_t, SYM_MAX_RANK> inner{};
    int32_t n_inner = 0;
    std::array<int64_t, SYM_MAX_RANK> shape{};
    std::array<int64_t, SYM_MAX_RANK> stride{};
    int64_t offset = 0;      // element offset of entry (0,..,0)
    int64_t size = 0;
    int32_t sector = -1;
};

struct Sector {
    int32_t label = 0;
    int64_t rows = 0, cols = 0;
    int64_t ld = 0;          // elements between consecutive stored rows
    int64_t offset = 0;      // element offset of the sector matrix
    std::vector<Tuple> row_tuples, col_tuples;
    std::vector<int64_t> row_off, col_off;
};

// Layout options beyond the ABI's packed sector-major layout, used only for
// the library's own fused workspaces.
struct LayoutOpts {
    bool trans = false;      // store each sector matrix transposed (cols x rows)
    int64_t ld_align = 1;    // leading dimension rounded up to this many elements
    int64_t base_align = 1;  // sector offsets rounded up to this many elements
};

struct Desc {
    int32_t group = SYM_U1, rank = 0, n_row = 0, tree = SYM_TREE_NONE, qtot = 0, dtype = SYM_F32;
    LayoutOpts opts;
    std::vector<Leg> legs;
    std::vector<Block> blocks;       // canonical order
    std::vector<Sector> sectors;     // ascending label
    int64_t numel = 0;               // elements the data spans (incl. padding)
    std::string key;                 // structural signature
    std::unordered_map<std::string, int32_t> block_index;  // label tuple (+internal) -> block

    int32_t find_block(const int32_t* labels, int32_t internal) const;
    // block with these labels and the intermediate spins of `like` (its
    // internal, or its CHAIN key)
    int32_t find_block(const int32_t* labels, const Block& like) const;
    int32_t find_block_inner(const int32_t* labels, const int32_t* inner, int32_t n_inner) const;
    int32_t find_sector(int32_t label) const;
};

using DescPtr = std::shared_ptr<const Desc>;

std::string label_key(const int32_t* labels, int n, int32_t internal);
std::string inner_key(const int32_t* labels, int n, const int32_t* inner, int n_inner);
DescPtr make_desc(int32_t group, const std::vector<Leg>& legs, int32_t n_row, int32_t tree,
                  int32_t qtot, int32_t dtype, const LayoutOpts& opts = LayoutOpts());
std::vector<Leg> permute_legs(const std::vector<Leg>& legs, const std::vector<int32_t>& perm);
size_t dtype_size(int32_t dtype);

// SU(2) fusion rule on doubled spins.
inline bool triangle(int a, int b, int c) {
    return (a + b + c) % 2 == 0 && c >= (a > b ? a - b : b - a) && c <= a + b;
}

// SU(2) CHAIN tree (tensors of any rank; section "Tree decompositions of
// SU(2)-invariant tensors", eq:datastruct, with left-associative fusion
// trees): the incoming legs, in leg order c_0, c_1, ..., are fused as
// (c_0, c_1 -> a_1), (a_1, c_2 -> a_2), ... to a total spin J, the outgoing
// legs d_0, d_1, ... likewise (b_1, b_2, ...) to the same J.  An empty chain
// has total 0.  A coupled sequence is (a_0 = j_{c_0}, a_1, .., a_{n-1} = J).
// The key of a block lists its free intermediate spins:
// (a_1 .. a_{n-2}, J if both chains have two legs or more, b_1 .. b_{m-2}).
using Seq = std::vector<int32_t>;
std::vector<Seq> chain_sequences(const std::vector<int32_t>& spins);
inline int32_t chain_total(const Seq& s) { return s.empty() ? 0 : s.back(); }
std::vector<int32_t> chain_key(const Seq& a, const Seq& b);
struct ChainBlock {
    Seq a, b;                     // coupled sequences of the incoming and outgoing chains
    std::vector<int32_t> key;
};
// every CHAIN block of one label tuple (labels in leg order), sorted by key
std::vector<ChainBlock> chain_blocks(const std::vector<int32_t>& arrows, const int32_t* labels, int rank);
// Recoupling coefficient F^{D E}_{A B C J} (eq:sixj), doubled spins.
double fmove_coeff(int tA, int tB, int tC, int tJ, int tD, int tE);
double sixj(int a, int b, int c, int d, int e, int f);

// Rank-4 SU(2) PERMUTE with recoupling and reversal (newtree.cpp).  A state
// is a tree kind (0 OPERATOR, 1 LEFT, 2 RIGHT) with the input leg in each
// slot; moves[k] takes states[k] to states[k + 1].
struct TreeState {
    int kind;
    std::array<int, 4> slot;
};
struct TreeMoves {
    std::vector<TreeState> states;
    std::vector<int> moves;
};
// Shortest sequence of moves from the tree tree_in on legs (0,1,2,3) to
// tree_out on legs (perm[0], .., perm[3]).
TreeMoves tree_moves(int32_t tree_in, const int32_t* perm, int32_t tree_out);
// Gamma of one label tuple (j[leg] = doubled spin of input leg leg): es and fs
// are the input's and output's intermediate spins, coef[f][e] row-major.
void tree_gamma(const TreeMoves& mv, const int32_t* j, std::vector<int32_t>& es, std::vector<int32_t>& fs,
                std::vector<double>& coef);

// Gamma of a PERMUTE with REVERSE between CHAIN trees (newtree.cpp): input
// legs with arrows_in and doubled spins j; output leg i is input leg perm[i]
// with arrow arrows_out[i].  keys_in / keys_out: the blocks' keys in block
// order; coef[f * n + e] maps input block e to output block f.
void chain_gamma(int rank, const int32_t* arrows_in, const int32_t* perm, const int32_t* arrows_out,
                 const int32_t* j, std::vector<std::vector<int32_t>>& keys_in,
                 std::vector<std::vector<int32_t>>& keys_out, std::vector<double>& coef);

}  // namespace sym
