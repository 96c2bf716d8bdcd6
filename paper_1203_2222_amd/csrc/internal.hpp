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

// A tuple of labels on a subset of legs, with its degeneracy product.
struct Tuple {
    std::array<int32_t, SYM_MAX_RANK> lab{};
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
    int32_t internal = -1;   // SU(2) intermediate spin (doubled); -1 for U(1)
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
    int32_t find_sector(int32_t label) const;
};

using DescPtr = std::shared_ptr<const Desc>;

std::string label_key(const int32_t* labels, int n, int32_t internal);
DescPtr make_desc(int32_t group, const std::vector<Leg>& legs, int32_t n_row, int32_t tree,
                  int32_t qtot, int32_t dtype, const LayoutOpts& opts = LayoutOpts());
std::vector<Leg> permute_legs(const std::vector<Leg>& legs, const std::vector<int32_t>& perm);
size_t dtype_size(int32_t dtype);

// SU(2) fusion rule on doubled spins.
inline bool triangle(int a, int b, int c) {
    return (a + b + c) % 2 == 0 && c >= (a > b ? a - b : b - a) && c <= a + b;
}
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

}  // namespace sym
