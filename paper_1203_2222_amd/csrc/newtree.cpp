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
#include <algorithm>
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

// ---------------------------------------------------------------------------
// CHAIN trees of any rank (see internal.hpp): Gamma of a PERMUTE with
// REVERSE composed from four elementary moves on the two chains, each a
// sparse matrix on the basis of coupled sequences of one label tuple:
//
//   SWAP at the first node of a chain   (c0, c1 -> a1) -> (c1, c0 -> a1):
//                                       (-1)^(j0+j1-a1)                    eq:braid3
//   SWAP further up, positions i, i+1   F-move, swap at the new node,
//                                       inverse F-move:
//                                       sum_E F^{D E}_{A B C J} (-1)^(B+C-E) F^{D' E}_{A C B J}
//                                                                          eq:fmove2, eq:sixj
//   UNBEND: the last incoming leg c (node (A, c -> J)) becomes the last
//           outgoing one (node (J, c -> A)):  sqrt((2J+1)/(2A+1)) (-1)^(c+J-A)
//   BEND:   the last outgoing leg d (node (B, d -> J)) becomes the last
//           incoming one (node (J, d -> B)):  (-1)^(B+d-J) sqrt((2J+1)/(2B+1))
//                                                                          eq:cupj, eq:capj
//
// The bends are the rank-4 bend (sqrt((2e+1)/(2d+1)) for the first slot of
// a node, cup on an outgoing leg, cap on an incoming one) composed with the
// exchange that puts the leg in that slot.
namespace sym {
namespace {

struct ChainSt {
    std::vector<int> in, out;   // input leg ids, chain order
};

struct Basis {
    std::vector<std::pair<Seq, Seq>> el;
    std::map<std::pair<Seq, Seq>, int> index;
};

Basis chain_basis(const ChainSt& s, const int32_t* j) {
    std::vector<int32_t> si, so;
    for (int l : s.in) si.push_back(j[l]);
    for (int l : s.out) so.push_back(j[l]);
    Basis B;
    for (const Seq& a : chain_sequences(si))
        for (const Seq& b : chain_sequences(so))
            if (chain_total(a) == chain_total(b)) {
                B.index[{a, b}] = static_cast<int>(B.el.size());
                B.el.push_back({a, b});
            }
    return B;
}

double sgn(int twice) { return ((twice / 2) & 1) ? -1.0 : 1.0; }

// coefficient of the adjacent exchange at positions i >= 1 of a chain:
// ((A, B -> D), C -> J)  ->  ((A, C -> D'), B -> J)
double exchange(int A, int B, int C, int J, int D, int Dp) {
    double v = 0.0;
    const int lo = B > C ? B - C : C - B;
    for (int E = lo; E <= B + C; E += 2) {
        if (!triangle(A, E, J)) continue;
        v += fmove_coeff(A, B, C, J, D, E) * sgn(B + C - E) * fmove_coeff(A, C, B, J, Dp, E);
    }
    return v;
}

// one move applied to the matrix M (rows: basis of the current state, columns: input basis)
void apply(int kind, int pos, ChainSt& st, Basis& cur, std::vector<std::vector<double>>& M, const int32_t* j) {
    ChainSt nx = st;
    if (kind == 0) std::swap(nx.in[static_cast<size_t>(pos)], nx.in[static_cast<size_t>(pos + 1)]);
    else if (kind == 1) std::swap(nx.out[static_cast<size_t>(pos)], nx.out[static_cast<size_t>(pos + 1)]);
    else if (kind == 2) { nx.out.push_back(nx.in.back()); nx.in.pop_back(); }   // UNBEND
    else { nx.in.push_back(nx.out.back()); nx.out.pop_back(); }                  // BEND
    Basis nb = chain_basis(nx, j);
    if (nb.el.size() != cur.el.size()) throw Error(SYM_E_MISMATCH, "chain moves change the multiplicity");
    const size_t cols = M.empty() ? 0 : M[0].size();
    std::vector<std::vector<double>> R(nb.el.size(), std::vector<double>(cols, 0.0));
    auto add = [&](const Seq& a, const Seq& b, double coef, size_t from) {
        if (coef == 0.0) return;
        auto it = nb.index.find({a, b});
        if (it == nb.index.end()) throw Error(SYM_E_MISMATCH, "chain move leaves the basis");
        std::vector<double>& row = R[static_cast<size_t>(it->second)];
        for (size_t c = 0; c < cols; ++c) row[c] += coef * M[from][c];
    };
    for (size_t q = 0; q < cur.el.size(); ++q) {
        const Seq& a = cur.el[q].first;
        const Seq& b = cur.el[q].second;
        if (kind == 0 || kind == 1) {
            const Seq& s = kind == 0 ? a : b;
            const std::vector<int>& legs = kind == 0 ? st.in : st.out;
            const int B = j[legs[static_cast<size_t>(pos)]], C = j[legs[static_cast<size_t>(pos + 1)]];
            if (pos == 0) {
                Seq t = s;
                t[0] = C;
                const double coef = sgn(B + C - s[1]);
                if (kind == 0) add(t, b, coef, q);
                else add(a, t, coef, q);
            } else {
                const int A = s[static_cast<size_t>(pos - 1)], D = s[static_cast<size_t>(pos)],
                          J = s[static_cast<size_t>(pos + 1)];
                const int lo = A > C ? A - C : C - A;
                for (int Dp = lo; Dp <= A + C; Dp += 2) {
                    if (!triangle(Dp, B, J)) continue;
                    Seq t = s;
                    t[static_cast<size_t>(pos)] = Dp;
                    const double coef = exchange(A, B, C, J, D, Dp);
                    if (kind == 0) add(t, b, coef, q);
                    else add(a, t, coef, q);
                }
            }
        } else if (kind == 2) {
            const int c = j[st.in.back()];
            const int J = a.back();
            const int A = a.size() >= 2 ? a[a.size() - 2] : 0;
            Seq a2(a.begin(), a.end() - 1), b2 = b;
            b2.push_back(A);
            add(a2, b2, std::sqrt((J + 1.0) / (A + 1.0)) * sgn(c + J - A), q);
        } else {
            const int d = j[st.out.back()];
            const int J = b.back();
            const int Bq = b.size() >= 2 ? b[b.size() - 2] : 0;
            Seq b2(b.begin(), b.end() - 1), a2 = a;
            a2.push_back(Bq);
            add(a2, b2, sgn(Bq + d - J) * std::sqrt((J + 1.0) / (Bq + 1.0)), q);
        }
    }
    M.swap(R);
    cur = std::move(nb);
    st = nx;
}

}  // namespace

void chain_gamma(int rank, const int32_t* arrows_in, const int32_t* perm, const int32_t* arrows_out,
                 const int32_t* j, std::vector<std::vector<int32_t>>& keys_in,
                 std::vector<std::vector<int32_t>>& keys_out, std::vector<double>& coef) {
    ChainSt st, goal;
    for (int l = 0; l < rank; ++l) (arrows_in[l] == SYM_IN ? st.in : st.out).push_back(l);
    for (int i = 0; i < rank; ++i) (arrows_out[i] == SYM_IN ? goal.in : goal.out).push_back(perm[i]);
    Basis cur = chain_basis(st, j);
    // the input basis in block order (by key)
    std::vector<size_t> order(cur.el.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) {
        return chain_key(cur.el[x].first, cur.el[x].second) < chain_key(cur.el[y].first, cur.el[y].second);
    });
    const size_t n = cur.el.size();
    std::vector<std::vector<double>> M(n, std::vector<double>(n, 0.0));
    for (size_t c = 0; c < n; ++c) M[order[c]][c] = 1.0;   // column c = input block c
    keys_in.clear();
    for (size_t c = 0; c < n; ++c) keys_in.push_back(chain_key(cur.el[order[c]].first, cur.el[order[c]].second));
    auto want_in = [&](int l) { return std::find(goal.in.begin(), goal.in.end(), l) != goal.in.end(); };
    // legs that change chain: to the end of their chain, then across
    for (bool moved = true; moved;) {
        moved = false;
        for (size_t p = 0; p < st.in.size(); ++p)
            if (!want_in(st.in[p])) {
                for (size_t q = p; q + 1 < st.in.size(); ++q) apply(0, static_cast<int>(q), st, cur, M, j);
                apply(2, 0, st, cur, M, j);
                moved = true;
                break;
            }
    }
    for (bool moved = true; moved;) {
        moved = false;
        for (size_t p = 0; p < st.out.size(); ++p)
            if (want_in(st.out[p])) {
                for (size_t q = p; q + 1 < st.out.size(); ++q) apply(1, static_cast<int>(q), st, cur, M, j);
                apply(3, 0, st, cur, M, j);
                moved = true;
                break;
            }
    }
    // order each chain as the goal (bubble sort by adjacent exchanges)
    for (int side = 0; side < 2; ++side) {
        std::vector<int>& ch = side == 0 ? st.in : st.out;
        const std::vector<int>& g = side == 0 ? goal.in : goal.out;
        if (ch.size() != g.size()) throw Error(SYM_E_MISMATCH, "chains do not reach the goal");
        std::map<int, size_t> rank_of;
        for (size_t i = 0; i < g.size(); ++i) rank_of[g[i]] = i;
        for (size_t pass = 0; pass < ch.size(); ++pass)
            for (size_t q = 0; q + 1 < ch.size(); ++q)
                if (rank_of[ch[q]] > rank_of[ch[q + 1]]) apply(side, static_cast<int>(q), st, cur, M, j);
    }
    // output basis in block order
    std::vector<size_t> oorder(cur.el.size());
    for (size_t i = 0; i < oorder.size(); ++i) oorder[i] = i;
    std::sort(oorder.begin(), oorder.end(), [&](size_t x, size_t y) {
        return chain_key(cur.el[x].first, cur.el[x].second) < chain_key(cur.el[y].first, cur.el[y].second);
    });
    keys_out.clear();
    coef.assign(n * n, 0.0);
    for (size_t r = 0; r < n; ++r) {
        keys_out.push_back(chain_key(cur.el[oorder[r]].first, cur.el[oorder[r]].second));
        for (size_t c = 0; c < n; ++c) coef[r * n + c] = M[oorder[r]][c];
    }
}

}  // namespace sym
