// The matrix Gamma(tree, p, tree') of a rank-4 SU(2) PERMUTE (eq:Gamma,
// eq:permsu2), with the reversal of every leg whose arrow the target tree
// changes (section "Reversal of indices"), composed from elementary moves on
// the host in FP64:
//
//   exchange of the two legs of one node       swap factor (-1)^(a+b-c)   eq:braid3
//   F-move LEFT <-> RIGHT on the same slots    F^{e f}_{a b c d}          eq:fmove2, eq:sixj
//   exchange at the top node (RIGHT <-> LEFT)  swap factor (-1)^(a+f-d)   eq:braid3
//   bending the third leg of an OPERATOR       sqrt((2e+1)/(2d+1))        eq:cupj
//
// A state is a tree kind (OPERATOR {s0,s1->e} {s2,s3->e}; LEFT
// {s0,s1->e; e,s2->s3}; RIGHT {s1,s2->f; s0,f->s3}) plus the leg that sits in
// each slot.  Slot arrows are fixed by the kind (OPERATOR in,in,out,out;
// LEFT and RIGHT in,in,in,out), so a path from the input's state to the
// output's state reverses exactly the legs whose arrow differs.  The tensor
// is T = sum_e v[e] Q_e(state); a move maps v to the next state's vector.
//
// Bending: summing the outgoing slot-2 leg of an OPERATOR node {c,d->e}
// against the row index of cup_c gives sqrt((2e+1)/(2d+1)) times the LEFT
// node {e,c->d} (CG symmetry); the inverse bend (cap on the incoming slot-2
// leg of a LEFT tree) divides by the same factor, since cup_c cap_c = 1
// (eq:wiggle).
#include <array>
#include <cmath>
#include <deque>
#include <map>

#include "internal.hpp"

namespace sym {
namespace {

enum Kind { K_OP = 0, K_LEFT = 1, K_RIGHT = 2 };
enum Move { M_SWAP01, M_SWAP23, M_SWAP12, M_BEND, M_UNBEND, M_FMOVE, M_FMOVE_INV, M_ROT_LR, M_ROT_RL };

int kind_of(int32_t tree) {
    if (tree == SYM_TREE_OPERATOR) return K_OP;
    if (tree == SYM_TREE_LEFT) return K_LEFT;
    if (tree == SYM_TREE_RIGHT) return K_RIGHT;
    throw Error(SYM_E_ARG, "SU(2) tree must be OPERATOR, LEFT or RIGHT");
}

int code(const TreeState& s) { return ((s.kind * 4 + s.slot[0]) * 4 + s.slot[1]) * 4 + s.slot[2]; }

TreeState with(int kind, int a, int b, int c, int d) { return TreeState{kind, {a, b, c, d}}; }

std::vector<std::pair<int, TreeState>> neighbours(const TreeState& s) {
    const auto& t = s.slot;
    std::vector<std::pair<int, TreeState>> out;
    if (s.kind == K_OP) {
        out.push_back({M_SWAP01, with(K_OP, t[1], t[0], t[2], t[3])});
        out.push_back({M_SWAP23, with(K_OP, t[0], t[1], t[3], t[2])});
        out.push_back({M_BEND, with(K_LEFT, t[0], t[1], t[2], t[3])});
    } else if (s.kind == K_LEFT) {
        out.push_back({M_SWAP01, with(K_LEFT, t[1], t[0], t[2], t[3])});
        out.push_back({M_FMOVE, with(K_RIGHT, t[0], t[1], t[2], t[3])});
        out.push_back({M_ROT_LR, with(K_RIGHT, t[2], t[0], t[1], t[3])});
        out.push_back({M_UNBEND, with(K_OP, t[0], t[1], t[2], t[3])});
    } else {
        out.push_back({M_SWAP12, with(K_RIGHT, t[0], t[2], t[1], t[3])});
        out.push_back({M_FMOVE_INV, with(K_LEFT, t[0], t[1], t[2], t[3])});
        out.push_back({M_ROT_RL, with(K_LEFT, t[1], t[2], t[0], t[3])});
    }
    return out;
}

// Intermediate spins of a state for the leg spins j[leg], ascending.
std::vector<int32_t> spins(const TreeState& s, const int32_t* j) {
    const int a = j[s.slot[0]], b = j[s.slot[1]], c = j[s.slot[2]], d = j[s.slot[3]];
    std::vector<int32_t> out;
    const int hi = 2 * std::max(std::max(a, b), std::max(c, d)) + 1;
    for (int e = 0; e <= hi; ++e) {
        bool ok = false;
        if (s.kind == K_OP) ok = triangle(a, b, e) && triangle(c, d, e);
        else if (s.kind == K_LEFT) ok = triangle(a, b, e) && triangle(e, c, d);
        else ok = triangle(b, c, e) && triangle(a, e, d);
        if (ok) out.push_back(e);
    }
    return out;
}

double parity(int twice) { return ((twice / 2) & 1) ? -1.0 : 1.0; }

}  // namespace

TreeMoves tree_moves(int32_t tree_in, const int32_t* perm, int32_t tree_out) {
    TreeMoves mv;
    const TreeState start = with(kind_of(tree_in), 0, 1, 2, 3);
    const TreeState goal = with(kind_of(tree_out), perm[0], perm[1], perm[2], perm[3]);
    // breadth-first search over the 72 states; the first path found is a shortest one
    std::map<int, std::pair<int, TreeState>> prev;   // state -> (move, previous state)
    std::deque<TreeState> queue{start};
    prev[code(start)] = {-1, start};
    while (!queue.empty() && !prev.count(code(goal))) {
        const TreeState s = queue.front();
        queue.pop_front();
        for (const auto& [m, n] : neighbours(s)) {
            if (prev.count(code(n))) continue;
            prev[code(n)] = {m, s};
            queue.push_back(n);
        }
    }
    if (!prev.count(code(goal))) throw Error(SYM_E_UNSUPPORTED, "no sequence of tree moves reaches the target tree");
    std::vector<TreeState> states{goal};
    std::vector<int> moves;
    for (TreeState s = goal; code(s) != code(start);) {
        const auto& pm = prev[code(s)];
        moves.push_back(pm.first);
        s = pm.second;
        states.push_back(s);
    }
    mv.states.assign(states.rbegin(), states.rend());
    mv.moves.assign(moves.rbegin(), moves.rend());
    return mv;
}

void tree_gamma(const TreeMoves& mv, const int32_t* j, std::vector<int32_t>& es, std::vector<int32_t>& fs,
                std::vector<double>& coef) {
    es = spins(mv.states.front(), j);
    const size_t n = es.size();
    // M: rows = current state's spins, columns = input spins
    std::vector<double> m(n * n, 0.0);
    for (size_t i = 0; i < n; ++i) m[i * n + i] = 1.0;
    std::vector<int32_t> cur = es;
    for (size_t k = 0; k < mv.moves.size(); ++k) {
        const TreeState& s = mv.states[k];
        const std::vector<int32_t> nxt = spins(mv.states[k + 1], j);
        if (nxt.size() != n) throw Error(SYM_E_MISMATCH, "tree moves change the multiplicity");
        const int a = j[s.slot[0]], b = j[s.slot[1]], c = j[s.slot[2]], d = j[s.slot[3]];
        std::vector<double> step(n * n, 0.0);   // rows nxt, columns cur
        for (size_t r = 0; r < n; ++r) {
            for (size_t q = 0; q < n; ++q) {
                const int f = nxt[r], e = cur[q];
                double v = 0.0;
                switch (mv.moves[k]) {
                    case M_SWAP01: v = (f == e) ? parity(a + b - e) : 0.0; break;
                    case M_SWAP23: v = (f == e) ? parity(c + d - e) : 0.0; break;
                    case M_SWAP12: v = (f == e) ? parity(b + c - e) : 0.0; break;
                    case M_BEND: v = (f == e) ? std::sqrt((e + 1.0) / (d + 1.0)) : 0.0; break;
                    case M_UNBEND: v = (f == e) ? std::sqrt((d + 1.0) / (e + 1.0)) : 0.0; break;
                    case M_FMOVE: v = fmove_coeff(a, b, c, d, e, f); break;
                    case M_FMOVE_INV: v = fmove_coeff(a, b, c, d, f, e); break;
                    case M_ROT_LR: v = (f == e) ? parity(c + e - d) : 0.0; break;
                    case M_ROT_RL: v = (f == e) ? parity(a + e - d) : 0.0; break;
                    default: throw Error(SYM_E_ARG, "unknown tree move");
                }
                step[r * n + q] = v;
            }
        }
        std::vector<double> next(n * n, 0.0);
        for (size_t r = 0; r < n; ++r)
            for (size_t q = 0; q < n; ++q) {
                const double v = step[r * n + q];
                if (v == 0.0) continue;
                for (size_t c2 = 0; c2 < n; ++c2) next[r * n + c2] += v * m[q * n + c2];
            }
        m.swap(next);
        cur = nxt;
    }
    fs = cur;
    coef = m;
}

}  // namespace sym
