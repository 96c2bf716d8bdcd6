// C-ABI of the symtensor library: contexts, tensor handles, plan caches and
// the host side of permute / contract / backward / batched / graph calls.
#include <algorithm>
#include <limits>
#include <cstdio>
#include <deque>
#include <cstdlib>
#include <fstream>
#include <functional>
#include <sstream>

#include <hip/hip_runtime.h>

#include "plan.hpp"

using namespace sym;

namespace {

thread_local std::string g_last_error;

void set_error(const std::string& m) { g_last_error = m; }

#define HIP_CHECK(expr)                                                                    \
    do {                                                                                   \
        hipError_t _e = (expr);                                                            \
        if (_e != hipSuccess) throw Error(SYM_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename F>
int32_t guard(F&& f) {
    try {
        f();
        return SYM_OK;
    } catch (const Error& e) {
        set_error(e.what());
        return e.status;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return SYM_E_NOMEM;
    } catch (const std::exception& e) {
        set_error(e.what());
        return SYM_E_ARG;
    } catch (...) {   // nothing may cross the C-ABI as an exception
        set_error("unexpected exception");
        return SYM_E_ARG;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------

namespace {

// Buffer slots of a contraction launch.
constexpr int kSlotWsIn = 0;    // fused operands (compute dtype)
constexpr int kSlotWsOut = 1;   // GEMM outputs that still need a split (FP32)
constexpr int kSlotUser = 2;    // user tensors from here on
constexpr int kMaxBatch = (kMaxBufs - kSlotUser) / 3;

// A recoupling launched as part of a contraction (general SU(2) operands).
struct RcStep {
    RecoupleProgram prog;
    int in_slot = 0, out_slot = 0;
};

struct ContractPlan {
    int count = 0, compute = SYM_F32;
    CopyProgram fuse[2];   // by source dtype (F32, BF16) -> compute dtype
    GemmProgram gemm;
    CopyProgram split;     // FP32 -> FP32
    // general SU(2) contractions: operands recoupled into their GEMM forms
    // before the GEMM, results recoupled into C after it
    std::deque<RcStep> rc_pre, rc_post;
    // small Abelian contractions: the whole contraction as one launch
    // (fuse, GEMM and split programs empty)
    bool small = false;
    SmallProgram small_prog;
    // user slots whose tensors are operands already in their GEMM layout
    // (read in place; their data must be 256-byte aligned like a workspace)
    std::vector<int> direct_slots;
    DevMemPtr ws_in, ws_out;
    int64_t in_elems = 0, out_elems = 0;   // workspace sizes (compute dtype, FP32)
    int grid = 1;
    int64_t flops = 0;
    int requested_variant = -1;   // the variant asked for (the GEMM may run a fallback)
    // Plans of the no-alloc entry point: tables and workspaces live in the
    // fixed scratch array, which every such call reuses, so each launch first
    // repeats the table uploads and clears the fused-operand workspace.
    bool noalloc = false;
    Deferred staged;
};

struct BackwardPlan {
    CopyProgram copy_in[2];
    GemmProgram gemm;
    CopyProgram split;
    DevMemPtr ws_in, ws_out;
    int grid = 1;
};

struct PermutePlan {
    CopyProgram copy;
    RecoupleProgram recouple;
    bool is_recouple = false;
};

}  // namespace

struct sym_tensor {
    DescPtr d;
    void* data = nullptr;
};

// Block-wise SVD of one tensor structure: per-sector problems and FP64
// workspaces for the Jacobi vectors and rotations.
struct SvdPlan {
    std::vector<SvdProb> probs;
    std::vector<int32_t> pair_start;   // prefix sums of the block pairs per sector
    int32_t max_kp = 0;                // largest (even) block count
    int64_t u_elems = 0, s_elems = 0, vt_elems = 0, w_elems = 0, q_elems = 0;
    DevMemPtr d_probs, d_pairs, w, q, scale, shift, gpart, flag, lastrot;
    int32_t flag_host = 0;
    // polar mode: the products that turn U, S, Vt (kept in uv and s) into
    // W and P; tiles of the W products first
    std::vector<PolarGemm> pgemm;
    std::vector<PolarTile> ptiles;
    int32_t n_wtiles = 0;
    int64_t pw_elems = 0, pp_elems = 0;
    DevMemPtr uv, s, d_pgemm, d_ptiles;
};

// Plans kept alive for as long as a caller needs them (sym_hold_*): a graph
// captured outside the library replays kernels that read a plan's device
// tables and write its workspaces, so those must outlive any change to the
// context's caches.
struct HoldSet {
    std::mutex mu;
    std::vector<std::shared_ptr<const void>> plans;
    void add(const std::shared_ptr<const void>& p) {
        std::lock_guard<std::mutex> lk(mu);
        for (const auto& q : plans)
            if (q == p) return;
        plans.push_back(p);
    }
};

struct sym_hold {
    std::shared_ptr<HoldSet> set;
};

struct sym_ctx {
    sym_alloc_fn alloc = nullptr;
    sym_free_fn free_fn = nullptr;
    void* user = nullptr;
    std::mutex mu;   // plan caches and the active hold set
    std::unordered_map<std::string, std::shared_ptr<ContractPlan>> contract_plans;
    std::unordered_map<std::string, std::shared_ptr<ContractPlan>> noalloc_plans;
    std::unordered_map<std::string, std::shared_ptr<BackwardPlan>> backward_plans;
    std::unordered_map<std::string, std::shared_ptr<PermutePlan>> permute_plans;
    std::unordered_map<std::string, std::shared_ptr<SvdPlan>> svd_plans;
    std::shared_ptr<HoldSet> hold;
    std::mutex tmu;   // tile choice, tuner results and timing events
    int variant[2] = {-1, -1};
    int n_cu = 0;
    bool timing = false;
    bool events_ready = false;
    hipEvent_t ev[4] = {};
    std::unordered_map<std::string, int> tuned;   // plan key hash -> variant
    // The plans of the latest single contractions, found by the identity of
    // their descriptors (held here, so their addresses stay unique) without
    // building the structural key; cleared (under mu) whenever a cached
    // contraction plan may change: a new plan, a tuning, a clear, a forced
    // tile variant.
    struct Recent {
        DescPtr a, b, c;
        int32_t n = -1, compute = -1;
        std::array<int32_t, SYM_MAX_RANK> axa{}, axb{};
        std::shared_ptr<ContractPlan> plan;
    };
    std::array<Recent, 8> recent;
    int recent_next = 0;
    void forget_recent() {
        for (auto& r : recent) r = Recent();
    }

    // record a plan in the active hold set, if any
    void note(const std::shared_ptr<const void>& plan) {
        std::shared_ptr<HoldSet> h;
        {
            std::lock_guard<std::mutex> lk(mu);
            h = hold;
        }
        if (h) h->add(plan);
    }
    bool timing_on() {
        std::lock_guard<std::mutex> lk(tmu);
        return timing;
    }

    Allocator allocator() {
        return [this](size_t bytes) -> DevMemPtr {
            auto m = std::make_shared<DevMem>();
            const size_t b = std::max<size_t>(bytes, 256);
            if (alloc) {
                m->ptr = alloc(b, user);
                sym_free_fn f = free_fn;
                void* u = user;
                m->release = [f, u](void* p) {
                    if (f) f(p, u);
                };
            } else {
                void* p = nullptr;
                if (hipMalloc(&p, b) != hipSuccess) p = nullptr;
                m->ptr = p;
                m->release = [](void* q) { (void)hipFree(q); };
            }
            if (!m->ptr) throw Error(SYM_E_NOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
            m->bytes = b;
            return m;
        };
    }

    int cus() {
        if (n_cu == 0) {
            int dev = 0;
            HIP_CHECK(hipGetDevice(&dev));
            HIP_CHECK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
            if (n_cu <= 0) n_cu = 1;
        }
        return n_cu;
    }

    void ensure_events() {
        std::lock_guard<std::mutex> lk(tmu);
        if (events_ready) return;
        for (auto& e : ev) HIP_CHECK(hipEventCreate(&e));
        events_ready = true;
    }
};

struct sym_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::shared_ptr<ContractPlan>> plans;   // one per chunk of 64 members
    // a contraction that is one launch of the small-contraction kernel is
    // replayed by launching that kernel with the arguments fixed at creation
    // (a graph launch costs more than the one kernel it would hold)
    bool direct = false;
    PtrTable table{};
};

namespace {

// A tensor with stored elements needs a buffer; one with none (no allowed
// block) may have none: no kernel reads or writes it.
bool has_data(const sym_tensor* t) { return t->data != nullptr || t->d->numel == 0; }

std::vector<Leg> read_legs(int32_t rank, const sym_leg* legs) {
    if (rank < 0 || rank > SYM_MAX_RANK) throw Error(SYM_E_ARG, "rank outside [0, SYM_MAX_RANK]");
    if (rank > 0 && !legs) throw Error(SYM_E_ARG, "legs is NULL");
    std::vector<Leg> out(static_cast<size_t>(rank));
    for (int i = 0; i < rank; ++i) {
        const sym_leg& l = legs[i];
        if (l.n < 0 || (l.n > 0 && (!l.label || !l.deg))) throw Error(SYM_E_ARG, "leg arrays are NULL");
        out[static_cast<size_t>(i)].label.assign(l.label, l.label + l.n);
        out[static_cast<size_t>(i)].deg.assign(l.deg, l.deg + l.n);
        out[static_cast<size_t>(i)].arrow = l.arrow;
    }
    return out;
}

struct PairInfo {
    std::vector<int32_t> fa, fb, axa, axb;
    std::vector<int32_t> perm_a, perm_b;   // A: fa ++ axa ; B: axb ++ fb
    bool su2_general = false;              // SU(2) outside the rank-4 operator form
};

PairInfo check_pair(const Desc& A, const Desc& B, int32_t n, const int32_t* axesA, const int32_t* axesB) {
    if (A.group != B.group) throw Error(SYM_E_ARG, "operands belong to different groups");
    if (n < 0 || n > A.rank || n > B.rank) throw Error(SYM_E_ARG, "bad number of contracted legs");
    if (n > 0 && (!axesA || !axesB)) throw Error(SYM_E_ARG, "axes are NULL");
    PairInfo p;
    std::vector<bool> ua(static_cast<size_t>(A.rank), false), ub(static_cast<size_t>(B.rank), false);
    for (int i = 0; i < n; ++i) {
        const int32_t a = axesA[i], b = axesB[i];
        if (a < 0 || a >= A.rank || b < 0 || b >= B.rank || ua[static_cast<size_t>(a)] || ub[static_cast<size_t>(b)])
            throw Error(SYM_E_ARG, "axes out of range or repeated");
        ua[static_cast<size_t>(a)] = ub[static_cast<size_t>(b)] = true;
        const Leg& la = A.legs[static_cast<size_t>(a)];
        const Leg& lb = B.legs[static_cast<size_t>(b)];
        if (!la.same_spectrum(lb)) throw Error(SYM_E_SPECTRUM, "contracted legs carry different spectra");
        if (la.arrow == lb.arrow) throw Error(SYM_E_ARROW, "contracted legs must have opposite arrows");
        p.axa.push_back(a);
        p.axb.push_back(b);
    }
    for (int i = 0; i < A.rank; ++i)
        if (!ua[static_cast<size_t>(i)]) p.fa.push_back(i);
    for (int i = 0; i < B.rank; ++i)
        if (!ub[static_cast<size_t>(i)]) p.fb.push_back(i);
    if (static_cast<int>(p.fa.size() + p.fb.size()) > SYM_MAX_RANK) throw Error(SYM_E_ARG, "result rank too large");
    p.perm_a = p.fa;
    p.perm_a.insert(p.perm_a.end(), p.axa.begin(), p.axa.end());
    p.perm_b = p.axb;
    p.perm_b.insert(p.perm_b.end(), p.fb.begin(), p.fb.end());
    if (A.group == SYM_SU2) {
        const bool fast = A.tree == SYM_TREE_OPERATOR && n == 2 && p.axa == std::vector<int32_t>{2, 3} &&
                          p.axb == std::vector<int32_t>{0, 1} &&
                          (B.tree == SYM_TREE_OPERATOR || B.tree == SYM_TREE_LEFT);
        if (!fast) {
            // the five steps on CHAIN trees: both operands recoupled into
            // their matrix forms, one GEMM per coupled spin, the product
            // recoupled into C
            auto chainlike = [](const Desc& d) {
                return d.tree == SYM_TREE_CHAIN || d.tree == SYM_TREE_OPERATOR || d.tree == SYM_TREE_LEFT;
            };
            if (!chainlike(A) || !chainlike(B))
                throw Error(SYM_E_UNSUPPORTED, "SU(2) contraction takes CHAIN, OPERATOR or LEFT tensors");
            if (n < 1 || p.fa.empty() || p.fb.empty())
                throw Error(SYM_E_UNSUPPORTED, "SU(2) contraction needs a contracted leg and a free leg on each side");
            p.su2_general = true;
        }
    }
    return p;
}

DescPtr result_desc(const Desc& A, const Desc& B, const PairInfo& p) {
    std::vector<Leg> legs;
    for (int32_t i : p.fa) legs.push_back(A.legs[static_cast<size_t>(i)]);
    for (int32_t i : p.fb) legs.push_back(B.legs[static_cast<size_t>(i)]);
    if (A.group == SYM_SU2 && p.su2_general)
        return make_desc(SYM_SU2, legs, static_cast<int32_t>(legs.size()), SYM_TREE_CHAIN, 0, SYM_F32);
    if (A.group == SYM_SU2)
        return make_desc(SYM_SU2, legs, 2, B.tree, 0, SYM_F32);
    return make_desc(A.group, legs, static_cast<int32_t>(p.fa.size()), SYM_TREE_NONE, combine_qtot(A.group, A.qtot, B.qtot),
                     SYM_F32);
}

// descriptor of A's legs (fa ++ axa) with |fa| row legs
DescPtr fused_a(const Desc& A, const PairInfo& p, int32_t dtype, bool trans) {
    return make_desc(A.group, permute_legs(A.legs, p.perm_a), static_cast<int32_t>(p.fa.size()), A.tree, A.qtot, dtype,
                     workspace_opts(dtype, trans));
}

// descriptor of B's legs (axb ++ fb) with |axb| row legs
DescPtr fused_b(const Desc& B, const PairInfo& p, int32_t dtype, bool trans) {
    return make_desc(B.group, permute_legs(B.legs, p.perm_b), static_cast<int32_t>(p.axb.size()), B.tree, B.qtot, dtype,
                     workspace_opts(dtype, trans));
}

// GEMM forms of a general SU(2) contraction (CHAIN trees): A' = A's free
// legs (incoming, rows) then its contracted legs (outgoing); B' = B's
// contracted legs (incoming, rows, in the order of the axes) then its free
// legs (arrows kept), stored transposed; C' = A's free legs (incoming, rows)
// then B's free legs.  The sector of A' and C' is the coupled spin of A's
// free legs, that of B' the coupled spin of the contracted legs, which the
// GEMM pairs (the Clebsch-Gordan chains of the contracted legs contract to
// the identity, eq:cgunitary).
struct Su2Forms {
    DescPtr ap, bp, cp;
};

Su2Forms su2_forms(const Desc& A, const Desc& B, const PairInfo& p, int32_t compute) {
    Su2Forms f;
    std::vector<Leg> la = permute_legs(A.legs, p.perm_a), lb = permute_legs(B.legs, p.perm_b), lc;
    for (size_t i = 0; i < la.size(); ++i) la[i].arrow = i < p.fa.size() ? SYM_IN : SYM_OUT;
    for (size_t i = 0; i < p.axb.size(); ++i) lb[i].arrow = SYM_IN;
    for (size_t i = 0; i < p.fa.size(); ++i) lc.push_back(la[i]);
    for (size_t i = p.axb.size(); i < lb.size(); ++i) lc.push_back(lb[i]);
    f.ap = make_desc(SYM_SU2, la, static_cast<int32_t>(p.fa.size()), SYM_TREE_CHAIN, 0, compute,
                     workspace_opts(compute, false));
    f.bp = make_desc(SYM_SU2, lb, static_cast<int32_t>(p.axb.size()), SYM_TREE_CHAIN, 0, compute,
                     workspace_opts(compute, true));
    f.cp = make_desc(SYM_SU2, lc, static_cast<int32_t>(p.fa.size()), SYM_TREE_CHAIN, 0, SYM_F32);
    return f;
}

std::vector<int32_t> identity(int n) {
    std::vector<int32_t> v(static_cast<size_t>(n));
    for (int i = 0; i < n; ++i) v[static_cast<size_t>(i)] = i;
    return v;
}

std::vector<int32_t> inverse(const std::vector<int32_t>& p) {
    std::vector<int32_t> q(p.size());
    for (size_t i = 0; i < p.size(); ++i) q[static_cast<size_t>(p[i])] = static_cast<int32_t>(i);
    return q;
}

// Equal tensors up to the padding and orientation of their sector matrices.
bool same_structure(const Desc& a, const Desc& b) {
    return a.group == b.group && a.rank == b.rank && a.n_row == b.n_row && a.tree == b.tree && a.qtot == b.qtot &&
           a.dtype == b.dtype && a.legs == b.legs;
}

// The layout C must have for the GEMM to write it directly.
bool gemm_can_write(const Desc& want, const Desc& c) {
    return c.dtype == SYM_F32 && !c.opts.trans && c.n_row == want.n_row && c.legs == want.legs &&
           c.tree == want.tree && c.qtot == want.qtot && c.group == want.group;
}

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// SYM_SPLIT=separate keeps the split of a canonical output as its own pass
// (instead of the GEMM epilogue), e.g. to time the two phases apart.
bool split_env_forced() {
    const char* v = std::getenv("SYM_SPLIT");
    return v && std::string(v) == "separate";
}

// Device side of a plan build: the table uploads (recorded by the programs'
// upload calls) and the clears of fused-operand workspaces (the GEMM kernels
// read whole 16-byte chunks past the last column of a row and rely on that
// padding being zero; nothing ever writes it after this clear) run in the
// order of the caller's stream, which is the order in which the context's
// allocator hands out memory; the build then waits for that stream alone,
// so a cached plan is ready for calls on any stream.  Plans are built outside
// stream capture.
struct BuildUploads {
    Deferred copies;
    std::vector<DevMemPtr> clears;
    DevMemPtr zeroed(const Allocator& alloc, size_t bytes) {
        DevMemPtr m = alloc(bytes);
        clears.push_back(m);
        return m;
    }
    void finish(hipStream_t s) {
        for (const DevMemPtr& m : clears) HIP_CHECK(launch_zero16(m->ptr, m->bytes, s));
        for (const HostCopy& c : copies) HIP_CHECK(hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, s));
        HIP_CHECK(hipStreamSynchronize(s));
    }
};

std::string axes_key(int32_t n, const int32_t* a, const int32_t* b) {
    std::ostringstream k;
    for (int i = 0; i < n; ++i) k << a[i] << ',' << b[i] << ';';
    return k.str();
}

int pick_variant(sym_ctx* ctx, int compute, const std::string& key) {
    std::lock_guard<std::mutex> lk(ctx->tmu);
    if (ctx->variant[compute] >= 0) return ctx->variant[compute];
    auto it = ctx->tuned.find(std::to_string(compute) + ":" + std::to_string(std::hash<std::string>{}(key)));
    if (it != ctx->tuned.end()) return it->second;
    return gemm_default_variant(compute);
}

std::string contract_key(int32_t count, const sym_tensor* const* A, const sym_tensor* const* B, int32_t n,
                         const int32_t* axA, const int32_t* axB, int32_t compute, sym_tensor* const* C,
                         std::vector<PairInfo>* infos) {
    if (compute != SYM_F32 && compute != SYM_BF16) throw Error(SYM_E_DTYPE, "compute must be F32 or BF16");
    if (count < 1 || count > kMaxBatch) throw Error(SYM_E_ARG, "batch size outside [1, 84]");
    std::ostringstream k;
    k << "C|" << compute << '|' << axes_key(n, axA, axB);
    for (int i = 0; i < count; ++i) {
        if (!A[i] || !B[i] || !C[i]) throw Error(SYM_E_ARG, "tensor handle is NULL");
        PairInfo p = check_pair(*A[i]->d, *B[i]->d, n, axA, axB);
        if (infos) infos->push_back(std::move(p));
        k << '#' << A[i]->d->key << '#' << B[i]->d->key << '#' << C[i]->d->key;
    }
    return k.str();
}

// Small Abelian contractions (at most kSmallFlops useful FLOPs over the batch)
// run as one launch that reads the operands' blocks in place.  SYM_SMALL=off
// sends them through the fuse / grouped GEMM / split path instead.
constexpr int64_t kSmallFlops = int64_t{1} << 25;

bool small_env_off() {
    const char* v = std::getenv("SYM_SMALL");
    return v && std::string(v) == "off";
}

// A group of a block's legs as one strided index (legs of extent 1 ignored):
// each leg's stride must be the next one's times its extent.
bool merge_legs(const Block& b, const std::vector<int32_t>& legs, int64_t& len, int64_t& stride) {
    std::vector<int32_t> g;
    for (int32_t l : legs)
        if (b.shape[static_cast<size_t>(l)] > 1) g.push_back(l);
    len = 1;
    stride = 0;
    for (size_t i = 0; i + 1 < g.size(); ++i)
        if (b.stride[static_cast<size_t>(g[i])] !=
            b.stride[static_cast<size_t>(g[i + 1])] * b.shape[static_cast<size_t>(g[i + 1])])
            return false;
    for (int32_t l : g) len *= b.shape[static_cast<size_t>(l)];
    if (!g.empty()) stride = b.stride[static_cast<size_t>(g.back())];
    return true;
}

bool fits32(int64_t x) { return x >= 0 && x < (int64_t{1} << 31); }

// Tasks and block pairs of member i; false when a block is not a strided
// matrix over its row and column legs or the work exceeds the budget.
bool add_small(const Desc& a, const Desc& b, const Desc& c, const PairInfo& p, int i, int count, SmallProgram& sp) {
    const int nfa = static_cast<int>(p.fa.size());
    std::vector<int32_t> crow, ccol;
    for (int l = 0; l < c.rank; ++l) (l < nfa ? crow : ccol).push_back(l);
    // A's blocks by the labels of their free legs
    std::map<std::vector<int32_t>, std::vector<int32_t>> a_by_free;
    for (size_t k = 0; k < a.blocks.size(); ++k) {
        std::vector<int32_t> f;
        for (int32_t l : p.fa) f.push_back(a.blocks[k].labels[static_cast<size_t>(l)]);
        a_by_free[f].push_back(static_cast<int32_t>(k));
    }
    for (const Block& cb : c.blocks) {
        int64_t M, N, crs, ccs;
        if (!merge_legs(cb, crow, M, crs) || !merge_legs(cb, ccol, N, ccs)) return false;
        if (!fits32(crs) || !fits32(ccs) || !fits32(M * N)) return false;
        const int32_t first = static_cast<int32_t>(sp.pairs.size());
        std::vector<int32_t> f(cb.labels.begin(), cb.labels.begin() + nfa);
        auto it = a_by_free.find(f);
        if (it != a_by_free.end())
            for (int32_t ai : it->second) {
                const Block& ab = a.blocks[static_cast<size_t>(ai)];
                int32_t bl[SYM_MAX_RANK];
                for (size_t k = 0; k < p.axb.size(); ++k) bl[p.axb[k]] = ab.labels[static_cast<size_t>(p.axa[k])];
                for (size_t k = 0; k < p.fb.size(); ++k) bl[p.fb[k]] = cb.labels[static_cast<size_t>(nfa) + k];
                const int32_t bi = b.find_block(bl, -1);
                if (bi < 0) continue;
                const Block& bb = b.blocks[static_cast<size_t>(bi)];
                int64_t Ma, Ka, ars, acs, Kb, Nb, brs, bcs;
                if (!merge_legs(ab, p.fa, Ma, ars) || !merge_legs(ab, p.axa, Ka, acs) ||
                    !merge_legs(bb, p.axb, Kb, brs) || !merge_legs(bb, p.fb, Nb, bcs))
                    return false;
                if (Ma != M || Nb != N || Ka != Kb) throw Error(SYM_E_MISMATCH, "block shapes disagree");
                if (!fits32(ars) || !fits32(acs) || !fits32(brs) || !fits32(bcs) || !fits32(Ka)) return false;
                SmallPair sp1{};
                sp1.a_off = ab.offset;
                sp1.b_off = bb.offset;
                sp1.a_rs = static_cast<int32_t>(ars);
                sp1.a_cs = static_cast<int32_t>(acs);
                sp1.b_rs = static_cast<int32_t>(brs);
                sp1.b_cs = static_cast<int32_t>(bcs);
                sp1.K = static_cast<int32_t>(Ka);
                sp1.a_buf = kSlotUser + i;
                sp1.b_buf = kSlotUser + count + i;
                sp.pairs.push_back(sp1);
                sp.flops += 2 * M * N * Ka;
                if (sp.flops > kSmallFlops) return false;
            }
        for (int64_t e0 = 0; e0 < M * N; e0 += kSmallTaskElems) {
            const int64_t e1 = std::min<int64_t>(M * N, e0 + kSmallTaskElems);
            SmallTask t{};
            t.c_off = cb.offset;
            t.c_rs = static_cast<int32_t>(crs);
            t.c_cs = static_cast<int32_t>(ccs);
            t.N = static_cast<int32_t>(N);
            t.e0 = static_cast<int32_t>(e0);
            t.e1 = static_cast<int32_t>(e1);
            t.pair_first = first;
            t.pair_count = static_cast<int32_t>(sp.pairs.size()) - first;
            t.c_buf = kSlotUser + 2 * count + i;
            sp.tasks.push_back(t);
        }
    }
    return true;
}

bool small_eligible(const Desc& a, const Desc& b, const Desc& c, int32_t compute) {
    return is_abelian(a.group) && a.group != SYM_Z2F && compute == SYM_F32 && a.dtype == SYM_F32 &&
           b.dtype == SYM_F32 && c.dtype == SYM_F32 && !a.opts.trans && !b.opts.trans && !c.opts.trans;
}

// Host part of a contraction plan: block copies, sector GEMMs, tile list and
// workspace sizes; no device memory is touched.
std::shared_ptr<ContractPlan> plan_contract_host(sym_ctx* ctx, int32_t count, const sym_tensor* const* A,
                                                 const sym_tensor* const* B, const std::vector<PairInfo>& infos,
                                                 int32_t compute, sym_tensor* const* C, int var) {
    auto plan = std::make_shared<ContractPlan>();
    plan->count = count;
    plan->compute = compute;
    plan->gemm.compute = compute;
    plan->fuse[0].src_dtype = SYM_F32;
    plan->fuse[1].src_dtype = SYM_BF16;
    plan->fuse[0].dst_dtype = plan->fuse[1].dst_dtype = compute;
    plan->split.src_dtype = plan->split.dst_dtype = SYM_F32;
    if (!small_env_off()) {
        bool ok = true;
        SmallProgram sp;
        for (int i = 0; i < count && ok; ++i) {
            const Desc& a = *A[i]->d;
            const Desc& b = *B[i]->d;
            const Desc& c = *C[i]->d;
            const PairInfo& p = infos[static_cast<size_t>(i)];
            DescPtr want_c = result_desc(a, b, p);
            if (c.group != want_c->group || c.legs != want_c->legs || c.qtot != want_c->qtot || c.dtype != SYM_F32)
                throw Error(SYM_E_MISMATCH, "C does not describe the contraction result");
            ok = small_eligible(a, b, c, compute) && add_small(a, b, c, p, i, count, sp);
        }
        if (ok) {
            plan->small = true;
            plan->small_prog = std::move(sp);
            plan->flops = plan->small_prog.flops;
            plan->requested_variant = var;
            plan->grid = 1;
            return plan;
        }
    }
    int64_t in_off = 0, out_off = 0;
    for (int i = 0; i < count; ++i) {
        const Desc& a = *A[i]->d;
        const Desc& b = *B[i]->d;
        const Desc& c = *C[i]->d;
        const PairInfo& p = infos[static_cast<size_t>(i)];
        DescPtr want_c = result_desc(a, b, p);
        if (c.group != want_c->group || c.legs != want_c->legs || c.qtot != want_c->qtot ||
            (c.group == SYM_SU2 && c.tree != want_c->tree) || c.dtype != SYM_F32)
            throw Error(SYM_E_MISMATCH, "C does not describe the contraction result");
        if (p.su2_general) {
            // BF16 compute: the recoupling of A and B writes their GEMM
            // forms rounded to BF16 (from FP32 or BF16 data); FP32 inputs
            // need FP32 compute
            if ((compute != SYM_F32 && compute != SYM_BF16) || (compute == SYM_F32 && (a.dtype != SYM_F32 ||
                                                                                     b.dtype != SYM_F32)))
                throw Error(SYM_E_DTYPE, "general SU(2) contractions of BF16 data need BF16 compute");
            const Su2Forms f = su2_forms(a, b, p, compute);
            const int64_t a_base = in_off;
            in_off = align_up(in_off + f.ap->numel, 64);
            const int64_t b_base = in_off;
            in_off = align_up(in_off + f.bp->numel, 64);
            const int64_t c_base = out_off;
            out_off = align_up(out_off + f.cp->numel, 64);
            std::vector<int32_t> cperm = identity(c.rank);
            plan->rc_pre.emplace_back();
            plan->rc_pre.back().prog.build(a, *f.ap, p.perm_a, 0, a_base);
            plan->rc_pre.back().in_slot = kSlotUser + i;
            plan->rc_pre.back().out_slot = kSlotWsIn;
            // A contracted pair whose A leg is incoming is reversed on both
            // sides (cap on A's leg, cup on B's); cap . cup^T = (-1)^(2j)
            // (eq:capj, eq:cupj), so B's coefficients take that sign back
            uint32_t sign_legs = 0;
            for (size_t k = 0; k < p.axb.size(); ++k)
                if (b.legs[static_cast<size_t>(p.axb[k])].arrow == SYM_OUT) sign_legs |= 1u << p.axb[k];
            plan->rc_pre.emplace_back();
            plan->rc_pre.back().prog.build(b, *f.bp, p.perm_b, 0, b_base, sign_legs);
            plan->rc_pre.back().in_slot = kSlotUser + count + i;
            plan->rc_pre.back().out_slot = kSlotWsIn;
            plan->gemm.add(*f.cp, *f.ap, *f.bp, kSlotWsOut, kSlotWsIn, kSlotWsIn, c_base, a_base, b_base);
            plan->rc_post.emplace_back();
            plan->rc_post.back().prog.build(*f.cp, c, cperm, c_base, 0);
            plan->rc_post.back().in_slot = kSlotWsOut;
            plan->rc_post.back().out_slot = kSlotUser + 2 * count + i;
            continue;
        }
        DescPtr af = fused_a(a, p, compute, false);
        DescPtr bf = fused_b(b, p, compute, true);   // stored N x K: K contiguous
        // an operand already in its GEMM layout (sym_contract_operand_output)
        // is read in place: no fuse, no workspace
        int64_t a_base = 0, b_base = 0;
        int a_slot = kSlotWsIn, b_slot = kSlotWsIn;
        if (a.key == af->key) {
            a_slot = kSlotUser + i;
            plan->direct_slots.push_back(a_slot);
        } else {
            a_base = in_off;
            in_off = align_up(in_off + af->numel, 64);
            plan->fuse[a.dtype == SYM_BF16 ? 1 : 0].add(a, *af, p.perm_a, kSlotUser + i, kSlotWsIn, 0, a_base);
        }
        if (b.key == bf->key) {
            b_slot = kSlotUser + count + i;
            plan->direct_slots.push_back(b_slot);
        } else {
            b_base = in_off;
            in_off = align_up(in_off + bf->numel, 64);
            plan->fuse[b.dtype == SYM_BF16 ? 1 : 0].add(b, *bf, p.perm_b, kSlotUser + count + i, kSlotWsIn, 0,
                                                        b_base);
        }
        if (gemm_can_write(*want_c, c)) {
            plan->gemm.add(c, *af, *bf, kSlotUser + 2 * count + i, a_slot, b_slot, 0, a_base, b_base);
        } else if (!split_env_forced() &&
                   plan->gemm.add_indirect(*want_c, c, *af, *bf, kSlotUser + 2 * count + i, a_slot, b_slot, a_base,
                                           b_base)) {
            // C is a canonical block list: the GEMM epilogue performs the split
        } else {
            const int64_t c_base = out_off;
            out_off = align_up(out_off + want_c->numel, 64);
            plan->gemm.add(*want_c, *af, *bf, kSlotWsOut, a_slot, b_slot, c_base, a_base, b_base);
            plan->split.add(*want_c, c, identity(c.rank), kSlotWsOut, kSlotUser + 2 * count + i, c_base, 0);
        }
    }
    plan->requested_variant = var;
    plan->grid = ctx->cus() * gemm_blocks_per_cu(compute, var);
    plan->gemm.finalize(var, plan->grid);
    plan->flops = plan->gemm.flops;
    for (auto& f : plan->fuse) f.finalize();
    plan->split.finalize();
    plan->in_elems = in_off;
    plan->out_elems = out_off;
    return plan;
}

std::shared_ptr<ContractPlan> build_contract_plan(sym_ctx* ctx, int32_t count, const sym_tensor* const* A,
                                                  const sym_tensor* const* B, int32_t n, const int32_t* axA,
                                                  const int32_t* axB, int32_t compute, sym_tensor* const* C,
                                                  std::string* key_out, int variant_override, hipStream_t stream) {
    std::vector<PairInfo> infos;
    const std::string key = contract_key(count, A, B, n, axA, axB, compute, C, &infos);
    if (key_out) *key_out = key;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->contract_plans.find(key);
        if (it != ctx->contract_plans.end() && variant_override < 0 &&
            it->second->requested_variant == pick_variant(ctx, compute, key))
            return it->second;
    }
    const int var = variant_override >= 0 ? variant_override : pick_variant(ctx, compute, key);
    auto plan = plan_contract_host(ctx, count, A, B, infos, compute, C, var);
    Allocator alloc = ctx->allocator();
    BuildUploads up;
    if (plan->in_elems) plan->ws_in = up.zeroed(alloc, static_cast<size_t>(plan->in_elems) * dtype_size(compute));
    if (plan->out_elems) plan->ws_out = alloc(static_cast<size_t>(plan->out_elems) * sizeof(float));
    for (auto& f : plan->fuse) f.upload(alloc, &up.copies);
    plan->gemm.upload(alloc, &up.copies);
    plan->split.upload(alloc, &up.copies);
    for (auto& r : plan->rc_pre) r.prog.upload(alloc, &up.copies);
    for (auto& r : plan->rc_post) r.prog.upload(alloc, &up.copies);
    if (plan->small) plan->small_prog.upload(alloc, &up.copies);
    up.finish(stream);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->contract_plans[key] = plan;
    ctx->forget_recent();
    return plan;
}

// Plan of the no-alloc entry point on the current device: the workspaces
// and every table are laid out back to back in that device's scratch array
// (256-byte aligned ranges); the uploads are recorded, to be repeated before
// each launch.  No device memory is allocated.
std::shared_ptr<ContractPlan> build_noalloc_plan(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                                                 const int32_t* axA, const int32_t* axB, int32_t compute,
                                                 sym_tensor* C) {
    std::vector<PairInfo> infos;
    const std::string key = contract_key(1, &A, &B, n, axA, axB, compute, &C, &infos);
    int dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    void* base = nullptr;
    HIP_CHECK(noalloc_scratch(&base));
    const std::string nkey = "N|" + std::to_string(dev) + '|' + key;
    const int var = pick_variant(ctx, compute, key);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->noalloc_plans.find(nkey);
        if (it != ctx->noalloc_plans.end() && it->second->requested_variant == var) return it->second;
    }
    auto plan = plan_contract_host(ctx, 1, &A, &B, infos, compute, &C, var);
    plan->noalloc = true;
    size_t used = 0;
    char* const b = static_cast<char*>(base);
    Allocator arena = [b, &used](size_t bytes) -> DevMemPtr {
        auto m = std::make_shared<DevMem>();   // no release: the array is never freed
        m->bytes = static_cast<size_t>(align_up(static_cast<int64_t>(std::max<size_t>(bytes, 256)), 256));
        m->ptr = b + used;
        used += m->bytes;
        return m;
    };
    if (plan->in_elems) plan->ws_in = arena(static_cast<size_t>(plan->in_elems) * dtype_size(compute));
    if (plan->out_elems) plan->ws_out = arena(static_cast<size_t>(plan->out_elems) * sizeof(float));
    for (auto& f : plan->fuse) f.upload(arena, &plan->staged);
    plan->gemm.upload(arena, &plan->staged);
    plan->split.upload(arena, &plan->staged);
    for (auto& r : plan->rc_pre) r.prog.upload(arena, &plan->staged);
    for (auto& r : plan->rc_post) r.prog.upload(arena, &plan->staged);
    if (plan->small) plan->small_prog.upload(arena, &plan->staged);
    if (used > kNoAllocScratchBytes)
        throw Error(SYM_E_UNSUPPORTED, "contraction needs " + std::to_string(used) +
                                           " bytes of workspace and tables; the no-alloc scratch holds " +
                                           std::to_string(kNoAllocScratchBytes));
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->noalloc_plans[nkey] = plan;
    return plan;
}

PtrTable contract_table(const ContractPlan& plan, const sym_tensor* const* A, const sym_tensor* const* B,
                        sym_tensor* const* C) {
    PtrTable t{};
    t.p[kSlotWsIn] = plan.ws_in ? plan.ws_in->ptr : nullptr;
    t.p[kSlotWsOut] = plan.ws_out ? plan.ws_out->ptr : nullptr;
    for (int i = 0; i < plan.count; ++i) {
        if (!has_data(A[i]) || !has_data(B[i]) || !has_data(C[i])) throw Error(SYM_E_ARG, "tensor has no data pointer");
        t.p[kSlotUser + i] = A[i]->data;
        t.p[kSlotUser + plan.count + i] = B[i]->data;
        t.p[kSlotUser + 2 * plan.count + i] = C[i]->data;
    }
    return t;
}

void run_contract_plan(sym_ctx* ctx, const ContractPlan& plan, const sym_tensor* const* A, const sym_tensor* const* B,
                       sym_tensor* const* C, hipStream_t s, bool allow_timing) {
    const PtrTable t = contract_table(plan, A, B, C);
    for (int slot : plan.direct_slots)
        if ((reinterpret_cast<uintptr_t>(t.p[slot]) & 255u) != 0)
            throw Error(SYM_E_ARG, "an operand in GEMM layout needs 256-byte aligned data");
    if (plan.noalloc) {
        // the scratch array holds whatever the last call on this device left
        for (const HostCopy& c : plan.staged)
            HIP_CHECK(hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, s));
        if (plan.ws_in) HIP_CHECK(launch_zero16(plan.ws_in->ptr, plan.ws_in->bytes, s));
    }
    const bool timing = allow_timing && ctx->timing_on();
    if (timing) {
        ctx->ensure_events();
        HIP_CHECK(hipEventRecord(ctx->ev[0], s));
    }
    for (const auto& f : plan.fuse) HIP_CHECK(f.launch(t, s));
    for (const auto& r : plan.rc_pre) HIP_CHECK(r.prog.launch(t, r.in_slot, r.out_slot, s));
    if (timing) HIP_CHECK(hipEventRecord(ctx->ev[1], s));
    if (plan.small) HIP_CHECK(plan.small_prog.launch(t, s));
    HIP_CHECK(plan.gemm.launch(t, plan.grid, s));
    if (timing) HIP_CHECK(hipEventRecord(ctx->ev[2], s));
    HIP_CHECK(plan.split.launch(t, s));
    for (const auto& r : plan.rc_post) HIP_CHECK(r.prog.launch(t, r.in_slot, r.out_slot, s));
    if (timing) HIP_CHECK(hipEventRecord(ctx->ev[3], s));
}

}  // namespace

// ---------------------------------------------------------------------------
// exports
// ---------------------------------------------------------------------------

extern "C" {

const char* sym_last_error(void) { return g_last_error.c_str(); }
const char* sym_version(void) { return "symtensor 0.1 (gfx950)"; }

int32_t sym_ctx_create(sym_alloc_fn alloc, sym_free_fn free_fn, void* user, sym_ctx** out) {
    return guard([&] {
        if (!out) throw Error(SYM_E_ARG, "out is NULL");
        if ((alloc == nullptr) != (free_fn == nullptr)) throw Error(SYM_E_ARG, "give both alloc and free, or neither");
        auto* c = new sym_ctx();
        c->alloc = alloc;
        c->free_fn = free_fn;
        c->user = user;
        if (const char* f = std::getenv("SYM_TUNE_CACHE")) {
            std::ifstream in(f);
            std::string k;
            int v;
            while (in >> k >> v) c->tuned[k] = v;
        }
        *out = c;
    });
}

void sym_ctx_destroy(sym_ctx* ctx) {
    if (!ctx) return;
    if (ctx->events_ready)
        for (auto& e : ctx->ev) (void)hipEventDestroy(e);
    delete ctx;
}

int32_t sym_ctx_clear(sym_ctx* ctx) {
    return guard([&] {
        if (!ctx) throw Error(SYM_E_ARG, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->contract_plans.clear();
        ctx->forget_recent();
        ctx->noalloc_plans.clear();
        ctx->backward_plans.clear();
        ctx->permute_plans.clear();
        ctx->svd_plans.clear();
    });
}

int32_t sym_hold_begin(sym_ctx* ctx, sym_hold** out) {
    return guard([&] {
        if (!ctx || !out) throw Error(SYM_E_ARG, "NULL argument");
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->hold) throw Error(SYM_E_ARG, "a hold is already collecting on this context");
        auto* h = new sym_hold();
        h->set = std::make_shared<HoldSet>();
        ctx->hold = h->set;
        *out = h;
    });
}

int32_t sym_hold_end(sym_ctx* ctx) {
    return guard([&] {
        if (!ctx) throw Error(SYM_E_ARG, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->hold.reset();
    });
}

int32_t sym_hold_count(const sym_hold* h, int64_t* n) {
    return guard([&] {
        if (!h || !n) throw Error(SYM_E_ARG, "NULL argument");
        std::lock_guard<std::mutex> lk(h->set->mu);
        *n = static_cast<int64_t>(h->set->plans.size());
    });
}

void sym_hold_destroy(sym_hold* h) { delete h; }

int32_t sym_tensor_create(sym_ctx* ctx, int32_t group, int32_t rank, const sym_leg* legs, int32_t n_row, int32_t tree,
                          int32_t qtot, int32_t dtype, void* data, sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!out) throw Error(SYM_E_ARG, "out is NULL");
        auto* t = new sym_tensor();
        try {
            t->d = make_desc(group, read_legs(rank, legs), n_row, tree, qtot, dtype);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *out = t;
    });
}

void sym_tensor_destroy(sym_tensor* t) { delete t; }

int32_t sym_tensor_set_data(sym_tensor* t, void* data) {
    return guard([&] {
        if (!t) throw Error(SYM_E_ARG, "tensor is NULL");
        t->data = data;
    });
}

int32_t sym_tensor_numel(const sym_tensor* t, int64_t* numel) {
    return guard([&] {
        if (!t || !numel) throw Error(SYM_E_ARG, "NULL argument");
        *numel = t->d->numel;
    });
}

int32_t sym_tensor_num_blocks(const sym_tensor* t, int64_t* n) {
    return guard([&] {
        if (!t || !n) throw Error(SYM_E_ARG, "NULL argument");
        *n = static_cast<int64_t>(t->d->blocks.size());
    });
}

int32_t sym_tensor_num_sectors(const sym_tensor* t, int64_t* n) {
    return guard([&] {
        if (!t || !n) throw Error(SYM_E_ARG, "NULL argument");
        *n = static_cast<int64_t>(t->d->sectors.size());
    });
}

int32_t sym_tensor_block_info(const sym_tensor* t, int64_t i, int32_t* labels, int32_t* internal, int64_t* offset,
                              int64_t* shape, int64_t* strides) {
    return guard([&] {
        if (!t) throw Error(SYM_E_ARG, "tensor is NULL");
        if (i < 0 || i >= static_cast<int64_t>(t->d->blocks.size())) throw Error(SYM_E_ARG, "block index out of range");
        const Block& b = t->d->blocks[static_cast<size_t>(i)];
        for (int l = 0; l < t->d->rank; ++l) {
            if (labels) labels[l] = b.labels[static_cast<size_t>(l)];
            if (shape) shape[l] = b.shape[static_cast<size_t>(l)];
            if (strides) strides[l] = b.stride[static_cast<size_t>(l)];
        }
        if (internal) *internal = b.internal;
        if (offset) *offset = b.offset;
    });
}

int32_t sym_tensor_block_inner(const sym_tensor* t, int64_t i, int32_t* inner, int32_t* n_inner) {
    return guard([&] {
        if (!t || !n_inner) throw Error(SYM_E_ARG, "NULL argument");
        if (i < 0 || i >= static_cast<int64_t>(t->d->blocks.size())) throw Error(SYM_E_ARG, "block index out of range");
        const Block& b = t->d->blocks[static_cast<size_t>(i)];
        *n_inner = b.n_inner;
        if (inner)
            for (int k = 0; k < b.n_inner; ++k) inner[k] = b.inner[static_cast<size_t>(k)];
    });
}

int32_t sym_tensor_sector_info(const sym_tensor* t, int64_t i, int32_t* label, int64_t* rows, int64_t* cols,
                               int64_t* offset) {
    return guard([&] {
        if (!t) throw Error(SYM_E_ARG, "tensor is NULL");
        if (i < 0 || i >= static_cast<int64_t>(t->d->sectors.size())) throw Error(SYM_E_ARG, "sector index out of range");
        const Sector& s = t->d->sectors[static_cast<size_t>(i)];
        if (label) *label = s.label;
        if (rows) *rows = s.rows;
        if (cols) *cols = s.cols;
        if (offset) *offset = s.offset;
    });
}

// ----- permute / fuse / recouple -------------------------------------------

namespace {

struct PermuteSpec {
    std::vector<int32_t> perm;
    bool recouple = false;
};

PermuteSpec check_perm(const Desc& in, const int32_t* perm) {
    PermuteSpec s;
    if (in.rank > 0 && !perm) throw Error(SYM_E_ARG, "perm is NULL");
    std::vector<bool> seen(static_cast<size_t>(in.rank), false);
    for (int i = 0; i < in.rank; ++i) {
        const int32_t p = perm[i];
        if (p < 0 || p >= in.rank || seen[static_cast<size_t>(p)]) throw Error(SYM_E_ARG, "not a permutation");
        seen[static_cast<size_t>(p)] = true;
        s.perm.push_back(p);
    }
    if (in.group == SYM_SU2) {
        if (s.perm == identity(4)) return s;
        if (s.perm == std::vector<int32_t>{0, 2, 1, 3} && in.tree == SYM_TREE_LEFT) {
            s.recouple = true;
            return s;
        }
        throw Error(SYM_E_UNSUPPORTED, "SU(2) permutations: identity, or (0,2,1,3) of a LEFT-tree tensor");
    }
    return s;
}

DescPtr permute_result(const Desc& in, const PermuteSpec& s, int32_t n_row_out, int32_t dtype_out) {
    if (s.recouple) {
        if (n_row_out != 0 && n_row_out != 4) throw Error(SYM_E_UNSUPPORTED, "recoupled tensors use n_row 0 or 4");
        if (dtype_out != SYM_F32 || in.dtype != SYM_F32) throw Error(SYM_E_DTYPE, "recoupling works on FP32 data");
        return make_desc(SYM_SU2, permute_legs(in.legs, s.perm), n_row_out, SYM_TREE_RIGHT, 0, SYM_F32);
    }
    return make_desc(in.group, permute_legs(in.legs, s.perm), n_row_out, in.tree, in.qtot, dtype_out);
}

}  // namespace

int32_t sym_permute_fuse_output(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t n_row_out,
                                int32_t dtype_out, void* data, sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!in || !out) throw Error(SYM_E_ARG, "NULL argument");
        PermuteSpec s = check_perm(*in->d, perm);
        auto* t = new sym_tensor();
        try {
            t->d = permute_result(*in->d, s, n_row_out, dtype_out);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *out = t;
    });
}

int32_t sym_permute_fuse(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t n_row_out, sym_tensor* out,
                         void* stream) {
    return guard([&] {
        if (!ctx || !in || !out) throw Error(SYM_E_ARG, "NULL argument");
        PermuteSpec s = check_perm(*in->d, perm);
        if (!has_data(in) || !has_data(out)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        std::ostringstream k;
        k << "P|" << in->d->key << '|' << out->d->key << '|' << n_row_out << '|';
        for (int32_t p : s.perm) k << p << ',';
        std::shared_ptr<PermutePlan> plan;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto it = ctx->permute_plans.find(k.str());
            if (it != ctx->permute_plans.end()) plan = it->second;
        }
        if (!plan) {
            // validated once per structure; a cached plan implies the same check passed
            DescPtr want = permute_result(*in->d, s, n_row_out, out->d->dtype);
            // out may carry a padded or transposed layout (an operand made by
            // sym_contract_operand_output): the copy writes its blocks wherever
            // the layout puts them
            if (!same_structure(*want, *out->d))
                throw Error(SYM_E_MISMATCH, "out does not describe the permuted tensor");
            if (out->d->opts.trans && s.recouple) throw Error(SYM_E_UNSUPPORTED, "no recoupling into a transposed layout");
            plan = std::make_shared<PermutePlan>();
            Allocator alloc = ctx->allocator();
            BuildUploads up;
            if (s.recouple) {
                plan->is_recouple = true;
                plan->recouple.build(*in->d, *out->d, s.perm);
                plan->recouple.upload(alloc, &up.copies);
            } else {
                plan->copy.src_dtype = in->d->dtype;
                plan->copy.dst_dtype = out->d->dtype;
                plan->copy.add(*in->d, *out->d, s.perm, 0, 1);
                plan->copy.finalize();
                plan->copy.upload(alloc, &up.copies);
            }
            up.finish(static_cast<hipStream_t>(stream));
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->permute_plans[k.str()] = plan;
        }
        ctx->note(plan);
        PtrTable t{};
        t.p[0] = in->data;
        t.p[1] = out->data;
        hipStream_t st = static_cast<hipStream_t>(stream);
        if (plan->is_recouple) HIP_CHECK(plan->recouple.launch(t, 0, 1, st));
        else HIP_CHECK(plan->copy.launch(t, st));
    });
}

// ----- SU(2) PERMUTE to a chosen tree, with REVERSE --------------------------------

namespace {

std::vector<int32_t> check_tree_perm(const Desc& in, const int32_t* perm, int32_t tree_out) {
    if (in.group != SYM_SU2)
        throw Error(SYM_E_UNSUPPORTED, "sym_permute_tree acts on SU(2) tensors (Abelian ones use sym_permute_fuse)");
    if (tree_out != SYM_TREE_OPERATOR && tree_out != SYM_TREE_LEFT && tree_out != SYM_TREE_RIGHT)
        throw Error(SYM_E_ARG, "tree_out must be OPERATOR, LEFT or RIGHT");
    if (!perm) throw Error(SYM_E_ARG, "perm is NULL");
    std::vector<int32_t> p(perm, perm + 4);
    std::vector<bool> seen(4, false);
    for (int32_t v : p) {
        if (v < 0 || v >= 4 || seen[static_cast<size_t>(v)]) throw Error(SYM_E_ARG, "not a permutation");
        seen[static_cast<size_t>(v)] = true;
    }
    return p;
}

DescPtr tree_result(const Desc& in, const std::vector<int32_t>& perm, int32_t tree_out, int32_t n_row_out) {
    if (in.dtype != SYM_F32) throw Error(SYM_E_DTYPE, "recoupling works on FP32 data");
    static const int32_t op_arrows[4] = {SYM_IN, SYM_IN, SYM_OUT, SYM_OUT};
    static const int32_t fuse_arrows[4] = {SYM_IN, SYM_IN, SYM_IN, SYM_OUT};
    const int32_t* arrows = tree_out == SYM_TREE_OPERATOR ? op_arrows : fuse_arrows;
    std::vector<Leg> legs = permute_legs(in.legs, perm);
    for (size_t i = 0; i < 4; ++i) legs[i].arrow = arrows[i];
    return make_desc(SYM_SU2, legs, n_row_out, tree_out, 0, SYM_F32);
}

}  // namespace

int32_t sym_permute_tree_output(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t tree_out,
                                int32_t n_row_out, void* data, sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!in || !out) throw Error(SYM_E_ARG, "NULL argument");
        const std::vector<int32_t> p = check_tree_perm(*in->d, perm, tree_out);
        auto* t = new sym_tensor();
        try {
            t->d = tree_result(*in->d, p, tree_out, n_row_out);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *out = t;
    });
}

int32_t sym_permute_tree(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t tree_out,
                         int32_t n_row_out, sym_tensor* out, void* stream) {
    return guard([&] {
        if (!ctx || !in || !out) throw Error(SYM_E_ARG, "NULL argument");
        const std::vector<int32_t> p = check_tree_perm(*in->d, perm, tree_out);
        if (!has_data(in) || !has_data(out)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        std::ostringstream k;
        k << "T|" << in->d->key << '|' << out->d->key << '|' << n_row_out << '|' << tree_out << '|';
        for (int32_t v : p) k << v << ',';
        std::shared_ptr<PermutePlan> plan;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto it = ctx->permute_plans.find(k.str());
            if (it != ctx->permute_plans.end()) plan = it->second;
        }
        if (!plan) {
            DescPtr want = tree_result(*in->d, p, tree_out, n_row_out);
            if (want->key != out->d->key) throw Error(SYM_E_MISMATCH, "out does not describe the permuted tensor");
            plan = std::make_shared<PermutePlan>();
            plan->is_recouple = true;
            plan->recouple.build(*in->d, *out->d, p);
            BuildUploads up;
            plan->recouple.upload(ctx->allocator(), &up.copies);
            up.finish(static_cast<hipStream_t>(stream));
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->permute_plans[k.str()] = plan;
        }
        ctx->note(plan);
        PtrTable t{};
        t.p[0] = in->data;
        t.p[1] = out->data;
        HIP_CHECK(plan->recouple.launch(t, 0, 1, static_cast<hipStream_t>(stream)));
    });
}

// ----- SU(2) PERMUTE / REVERSE onto CHAIN trees (any rank) -------------------------

namespace {

std::vector<int32_t> check_su2_chain_perm(const Desc& in, const int32_t* perm, const int32_t* arrows_out) {
    if (in.group != SYM_SU2) throw Error(SYM_E_UNSUPPORTED, "sym_su2_permute acts on SU(2) tensors");
    if (in.tree != SYM_TREE_CHAIN && in.tree != SYM_TREE_OPERATOR && in.tree != SYM_TREE_LEFT)
        throw Error(SYM_E_UNSUPPORTED, "sym_su2_permute takes CHAIN, OPERATOR or LEFT tensors");
    if (in.dtype != SYM_F32) throw Error(SYM_E_DTYPE, "recoupling works on FP32 data");
    if (!perm || !arrows_out) throw Error(SYM_E_ARG, "NULL argument");
    std::vector<int32_t> p(perm, perm + in.rank);
    std::vector<bool> seen(static_cast<size_t>(in.rank), false);
    for (int i = 0; i < in.rank; ++i) {
        if (p[static_cast<size_t>(i)] < 0 || p[static_cast<size_t>(i)] >= in.rank || seen[static_cast<size_t>(p[static_cast<size_t>(i)])])
            throw Error(SYM_E_ARG, "not a permutation");
        seen[static_cast<size_t>(p[static_cast<size_t>(i)])] = true;
        if (arrows_out[i] != SYM_IN && arrows_out[i] != SYM_OUT) throw Error(SYM_E_ARG, "arrow must be SYM_IN or SYM_OUT");
    }
    return p;
}

DescPtr su2_chain_result(const Desc& in, const std::vector<int32_t>& perm, const int32_t* arrows_out, int32_t n_row_out) {
    std::vector<Leg> legs = permute_legs(in.legs, perm);
    for (size_t i = 0; i < legs.size(); ++i) legs[i].arrow = arrows_out[i];
    return make_desc(SYM_SU2, legs, n_row_out, SYM_TREE_CHAIN, 0, SYM_F32);
}

}  // namespace

int32_t sym_su2_permute_output(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, const int32_t* arrows_out,
                               int32_t n_row_out, void* data, sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!in || !out) throw Error(SYM_E_ARG, "NULL argument");
        const std::vector<int32_t> p = check_su2_chain_perm(*in->d, perm, arrows_out);
        auto* t = new sym_tensor();
        try {
            t->d = su2_chain_result(*in->d, p, arrows_out, n_row_out);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *out = t;
    });
}

int32_t sym_su2_permute(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, const int32_t* arrows_out,
                        int32_t n_row_out, sym_tensor* out, void* stream) {
    return guard([&] {
        if (!ctx || !in || !out) throw Error(SYM_E_ARG, "NULL argument");
        const std::vector<int32_t> p = check_su2_chain_perm(*in->d, perm, arrows_out);
        if (!has_data(in) || !has_data(out)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        std::ostringstream k;
        k << "U|" << in->d->key << '|' << out->d->key << '|';
        for (int32_t v : p) k << v << ',';
        std::shared_ptr<PermutePlan> plan;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto it = ctx->permute_plans.find(k.str());
            if (it != ctx->permute_plans.end()) plan = it->second;
        }
        if (!plan) {
            DescPtr want = su2_chain_result(*in->d, p, arrows_out, n_row_out);
            if (want->key != out->d->key) throw Error(SYM_E_MISMATCH, "out does not describe the permuted tensor");
            plan = std::make_shared<PermutePlan>();
            plan->is_recouple = true;
            plan->recouple.build(*in->d, *out->d, p);
            BuildUploads up;
            plan->recouple.upload(ctx->allocator(), &up.copies);
            up.finish(static_cast<hipStream_t>(stream));
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->permute_plans[k.str()] = plan;
        }
        ctx->note(plan);
        PtrTable t{};
        t.p[0] = in->data;
        t.p[1] = out->data;
        HIP_CHECK(plan->recouple.launch(t, 0, 1, static_cast<hipStream_t>(stream)));
    });
}

// ----- SU(2) FUSE / SPLIT of two adjacent legs (CHAIN trees) --------------------------

namespace {

void check_fuse_legs(const Desc& d, int32_t leg) {
    if (d.group != SYM_SU2 || (d.tree != SYM_TREE_CHAIN && d.tree != SYM_TREE_OPERATOR && d.tree != SYM_TREE_LEFT))
        throw Error(SYM_E_UNSUPPORTED, "FUSE and SPLIT act on SU(2) CHAIN, OPERATOR or LEFT tensors");
    if (d.dtype != SYM_F32) throw Error(SYM_E_DTYPE, "FUSE and SPLIT work on FP32 data");
    if (leg < 0 || leg + 1 >= d.rank) throw Error(SYM_E_ARG, "leg and leg + 1 must be legs of the tensor");
}

DescPtr fused_desc(const Desc& in, int32_t leg, int32_t n_row_out) {
    check_fuse_legs(in, leg);
    const Leg& a = in.legs[static_cast<size_t>(leg)];
    const Leg& b = in.legs[static_cast<size_t>(leg + 1)];
    if (a.arrow != b.arrow) throw Error(SYM_E_ARROW, "fused legs must share their arrow");
    std::vector<Leg> legs;
    for (int l = 0; l < in.rank; ++l) {
        if (l == leg + 1) continue;
        legs.push_back(l == leg ? fuse_legs(a, b).leg : in.legs[static_cast<size_t>(l)]);
    }
    return make_desc(SYM_SU2, legs, n_row_out, SYM_TREE_CHAIN, 0, SYM_F32);
}

DescPtr split_desc(const Desc& in, int32_t leg, const Leg& a, const Leg& b, int32_t n_row_out) {
    if (in.group != SYM_SU2 || in.tree != SYM_TREE_CHAIN) throw Error(SYM_E_UNSUPPORTED, "SPLIT acts on CHAIN tensors");
    if (in.dtype != SYM_F32) throw Error(SYM_E_DTYPE, "FUSE and SPLIT work on FP32 data");
    if (leg < 0 || leg >= in.rank || in.rank + 1 > SYM_MAX_RANK) throw Error(SYM_E_ARG, "bad leg or rank");
    const Leg& f = in.legs[static_cast<size_t>(leg)];
    Leg la = a, lb = b;
    la.arrow = lb.arrow = f.arrow;
    const Leg fl = fuse_legs(la, lb).leg;
    if (fl.label != f.label || fl.deg != f.deg) throw Error(SYM_E_SPECTRUM, "the leg is not the fusion of the two legs");
    std::vector<Leg> legs;
    for (int l = 0; l < in.rank; ++l) {
        if (l == leg) {
            legs.push_back(la);
            legs.push_back(lb);
        } else {
            legs.push_back(in.legs[static_cast<size_t>(l)]);
        }
    }
    return make_desc(SYM_SU2, legs, n_row_out, SYM_TREE_CHAIN, 0, SYM_F32);
}

void run_fuse(sym_ctx* ctx, const sym_tensor* in, sym_tensor* out, int32_t leg, bool to_fused, const std::string& key,
              hipStream_t stream) {
    if (!has_data(in) || !has_data(out)) throw Error(SYM_E_ARG, "tensor has no data pointer");
    std::shared_ptr<PermutePlan> plan;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->permute_plans.find(key);
        if (it != ctx->permute_plans.end()) plan = it->second;
    }
    if (!plan) {
        plan = std::make_shared<PermutePlan>();
        plan->is_recouple = true;
        if (to_fused) plan->recouple.build_fuse(*in->d, *out->d, leg, true);
        else plan->recouple.build_fuse(*out->d, *in->d, leg, false);
        BuildUploads up;
        plan->recouple.upload(ctx->allocator(), &up.copies);
        up.finish(stream);
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->permute_plans[key] = plan;
    }
    ctx->note(plan);
    PtrTable t{};
    t.p[0] = in->data;
    t.p[1] = out->data;
    HIP_CHECK(plan->recouple.launch(t, 0, 1, stream));
}

}  // namespace

int32_t sym_su2_fuse_output(sym_ctx* ctx, const sym_tensor* in, int32_t leg, int32_t n_row_out, void* data,
                            sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!in || !out) throw Error(SYM_E_ARG, "NULL argument");
        auto* t = new sym_tensor();
        try {
            t->d = fused_desc(*in->d, leg, n_row_out);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *out = t;
    });
}

int32_t sym_su2_fuse(sym_ctx* ctx, const sym_tensor* in, int32_t leg, int32_t n_row_out, sym_tensor* out,
                     void* stream) {
    return guard([&] {
        if (!ctx || !in || !out) throw Error(SYM_E_ARG, "NULL argument");
        DescPtr want = fused_desc(*in->d, leg, n_row_out);
        if (want->key != out->d->key) throw Error(SYM_E_MISMATCH, "out does not describe the fused tensor");
        run_fuse(ctx, in, out, leg, true, "F|" + in->d->key + '|' + out->d->key + '|' + std::to_string(leg),
                 static_cast<hipStream_t>(stream));
    });
}

int32_t sym_su2_split_output(sym_ctx* ctx, const sym_tensor* in, int32_t leg, const sym_leg* legs2, int32_t n_row_out,
                             void* data, sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!in || !out || !legs2) throw Error(SYM_E_ARG, "NULL argument");
        const std::vector<Leg> two = read_legs(2, legs2);
        auto* t = new sym_tensor();
        try {
            t->d = split_desc(*in->d, leg, two[0], two[1], n_row_out);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *out = t;
    });
}

int32_t sym_su2_split(sym_ctx* ctx, const sym_tensor* in, int32_t leg, sym_tensor* out, void* stream) {
    return guard([&] {
        if (!ctx || !in || !out) throw Error(SYM_E_ARG, "NULL argument");
        if (out->d->rank != in->d->rank + 1 || leg < 0 || leg >= in->d->rank) throw Error(SYM_E_ARG, "bad leg or rank");
        DescPtr want = split_desc(*in->d, leg, out->d->legs[static_cast<size_t>(leg)],
                                  out->d->legs[static_cast<size_t>(leg + 1)], out->d->n_row);
        if (want->key != out->d->key) throw Error(SYM_E_MISMATCH, "out does not describe the split tensor");
        run_fuse(ctx, in, out, leg, false, "S|" + in->d->key + '|' + out->d->key + '|' + std::to_string(leg),
                 static_cast<hipStream_t>(stream));
    });
}

int32_t sym_tensor_leg(const sym_tensor* t, int32_t leg, int32_t cap, int32_t* n, int32_t* labels, int64_t* degs,
                       int32_t* arrow) {
    return guard([&] {
        if (!t || !n) throw Error(SYM_E_ARG, "NULL argument");
        if (leg < 0 || leg >= t->d->rank) throw Error(SYM_E_ARG, "leg out of range");
        const Leg& l = t->d->legs[static_cast<size_t>(leg)];
        *n = static_cast<int32_t>(l.label.size());
        if (arrow) *arrow = l.arrow;
        if (!labels && !degs) return;   // a query of *n
        if (*n > cap) throw Error(SYM_E_ARG, "capacity too small for the leg's labels");
        if (labels) std::copy(l.label.begin(), l.label.end(), labels);
        if (degs) std::copy(l.deg.begin(), l.deg.end(), degs);
    });
}

int32_t sym_su2_gamma(int32_t tree_in, const int32_t* perm, int32_t tree_out, const int32_t* spins, int32_t cap,
                      int32_t* n, int32_t* es, int32_t* fs, double* gamma) {
    return guard([&] {
        if (!perm || !spins || !n || !es || !fs || !gamma) throw Error(SYM_E_ARG, "NULL argument");
        std::vector<bool> seen(4, false);
        for (int i = 0; i < 4; ++i) {
            if (perm[i] < 0 || perm[i] >= 4 || seen[static_cast<size_t>(perm[i])]) throw Error(SYM_E_ARG, "not a permutation");
            seen[static_cast<size_t>(perm[i])] = true;
            if (spins[i] < 0) throw Error(SYM_E_ARG, "negative spin");
        }
        const TreeMoves mv = tree_moves(tree_in, perm, tree_out);
        std::vector<int32_t> e, f;
        std::vector<double> g;
        tree_gamma(mv, spins, e, f, g);
        const int32_t m = static_cast<int32_t>(e.size());
        if (m > cap) throw Error(SYM_E_ARG, "capacity too small for the intermediate spins");
        *n = m;
        std::copy(e.begin(), e.end(), es);
        std::copy(f.begin(), f.end(), fs);
        std::copy(g.begin(), g.end(), gamma);
    });
}

int32_t sym_su2_chain_gamma(int32_t rank, const int32_t* arrows_in, const int32_t* perm, const int32_t* arrows_out,
                            const int32_t* spins, int32_t cap, int32_t* n, int32_t* key_len_in, int32_t* key_len_out,
                            int32_t* keys_in, int32_t* keys_out, double* gamma) {
    return guard([&] {
        if (!arrows_in || !perm || !arrows_out || !spins || !n || !key_len_in || !key_len_out || !keys_in || !keys_out ||
            !gamma)
            throw Error(SYM_E_ARG, "NULL argument");
        if (rank < 1 || rank > SYM_MAX_RANK) throw Error(SYM_E_ARG, "rank outside [1, SYM_MAX_RANK]");
        std::vector<bool> seen(static_cast<size_t>(rank), false);
        for (int i = 0; i < rank; ++i) {
            if (perm[i] < 0 || perm[i] >= rank || seen[static_cast<size_t>(perm[i])]) throw Error(SYM_E_ARG, "not a permutation");
            seen[static_cast<size_t>(perm[i])] = true;
            if (spins[i] < 0) throw Error(SYM_E_ARG, "negative spin");
            if ((arrows_in[i] != SYM_IN && arrows_in[i] != SYM_OUT) || (arrows_out[i] != SYM_IN && arrows_out[i] != SYM_OUT))
                throw Error(SYM_E_ARG, "arrow must be SYM_IN or SYM_OUT");
        }
        std::vector<std::vector<int32_t>> ki, ko;
        std::vector<double> g;
        chain_gamma(rank, arrows_in, perm, arrows_out, spins, ki, ko, g);
        const int32_t m = static_cast<int32_t>(ki.size());
        if (m > cap) throw Error(SYM_E_ARG, "capacity too small for the blocks of this label tuple");
        *n = m;
        *key_len_in = m ? static_cast<int32_t>(ki[0].size()) : 0;
        *key_len_out = m ? static_cast<int32_t>(ko[0].size()) : 0;
        for (int32_t r = 0; r < m; ++r) {
            std::copy(ki[static_cast<size_t>(r)].begin(), ki[static_cast<size_t>(r)].end(), keys_in + r * *key_len_in);
            std::copy(ko[static_cast<size_t>(r)].begin(), ko[static_cast<size_t>(r)].end(), keys_out + r * *key_len_out);
        }
        std::copy(g.begin(), g.end(), gamma);
    });
}

// ----- contraction ------------------------------------------------------------

int32_t sym_contract_output(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n, const int32_t* axesA,
                            const int32_t* axesB, void* data, sym_tensor** C) {
    (void)ctx;
    return guard([&] {
        if (!A || !B || !C) throw Error(SYM_E_ARG, "NULL argument");
        PairInfo p = check_pair(*A->d, *B->d, n, axesA, axesB);
        auto* t = new sym_tensor();
        try {
            t->d = result_desc(*A->d, *B->d, p);
        } catch (...) {
            delete t;
            throw;
        }
        t->data = data;
        *C = t;
    });
}

int32_t sym_contract_operand_output(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                                    const int32_t* axesA, const int32_t* axesB, int32_t compute, int32_t which,
                                    void* data, sym_tensor** out) {
    (void)ctx;
    return guard([&] {
        if (!A || !B || !out) throw Error(SYM_E_ARG, "NULL argument");
        if (compute != SYM_F32 && compute != SYM_BF16) throw Error(SYM_E_DTYPE, "compute must be F32 or BF16");
        if (which != 0 && which != 1) throw Error(SYM_E_ARG, "which must be 0 (A) or 1 (B)");
        PairInfo p = check_pair(*A->d, *B->d, n, axesA, axesB);
        if (p.su2_general) throw Error(SYM_E_UNSUPPORTED, "general SU(2) contractions have no operand layout");
        DescPtr d = which == 0 ? fused_a(*A->d, p, compute, false) : fused_b(*B->d, p, compute, true);
        auto* t = new sym_tensor();
        t->d = std::move(d);
        t->data = data;
        *out = t;
    });
}

int32_t sym_contract_flops(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n, const int32_t* axesA,
                           const int32_t* axesB, int64_t* flops) {
    (void)ctx;
    return guard([&] {
        if (!A || !B || !flops) throw Error(SYM_E_ARG, "NULL argument");
        PairInfo p = check_pair(*A->d, *B->d, n, axesA, axesB);
        GemmProgram g;
        if (p.su2_general) {
            const Su2Forms f = su2_forms(*A->d, *B->d, p, SYM_F32);
            g.add(*f.cp, *f.ap, *f.bp, 0, 0, 0);
        } else {
            DescPtr c = result_desc(*A->d, *B->d, p);
            g.add(*c, *fused_a(*A->d, p, SYM_F32, false), *fused_b(*B->d, p, SYM_F32, true), 0, 0, 0);
        }
        *flops = g.flops;
    });
}

int32_t sym_contract_batched(sym_ctx* ctx, int32_t count, const sym_tensor* const* A, const sym_tensor* const* B,
                             int32_t n, const int32_t* axesA, const int32_t* axesB, int32_t compute,
                             sym_tensor* const* C, void* stream) {
    return guard([&] {
        if (!ctx || !A || !B || !C) throw Error(SYM_E_ARG, "NULL argument");
        if (count < 1) throw Error(SYM_E_ARG, "count must be >= 1");
        // every member is checked, and every chunk planned, before the first
        // launch, so a bad member leaves all outputs untouched (one chunk is
        // checked by its own plan lookup)
        if (count > 64)
            for (int32_t first = 0; first < count; first += 64)
                (void)contract_key(std::min<int32_t>(64, count - first), A + first, B + first, n, axesA, axesB,
                                   compute, C + first, nullptr);
        std::vector<std::shared_ptr<ContractPlan>> plans;
        for (int32_t first = 0; first < count; first += 64) {
            const int32_t m = std::min<int32_t>(64, count - first);
            plans.push_back(build_contract_plan(ctx, m, A + first, B + first, n, axesA, axesB, compute, C + first,
                                                nullptr, -1, static_cast<hipStream_t>(stream)));
            for (int32_t i = first; i < first + m; ++i)
                if (!has_data(A[i]) || !has_data(B[i]) || !has_data(C[i]))
                    throw Error(SYM_E_ARG, "tensor has no data pointer");
        }
        for (size_t c = 0; c < plans.size(); ++c) {
            const int32_t first = static_cast<int32_t>(c) * 64;
            ctx->note(plans[c]);
            run_contract_plan(ctx, *plans[c], A + first, B + first, C + first, static_cast<hipStream_t>(stream),
                              count <= 64);
        }
    });
}

int32_t sym_contract(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n, const int32_t* axesA,
                     const int32_t* axesB, int32_t compute, sym_tensor* C, void* stream) {
    return guard([&] {
        if (!ctx || !A || !B || !C) throw Error(SYM_E_ARG, "NULL argument");
        // a repeated call on the same handles' descriptors finds its plan
        // without rebuilding the structural key
        std::shared_ptr<ContractPlan> plan;
        const bool axes_ok = n >= 0 && n <= SYM_MAX_RANK && (n == 0 || (axesA && axesB));
        if (axes_ok) {
            std::lock_guard<std::mutex> lk(ctx->mu);
            for (const auto& r : ctx->recent)
                if (r.plan && r.a == A->d && r.b == B->d && r.c == C->d && r.n == n && r.compute == compute &&
                    std::equal(axesA, axesA + n, r.axa.begin()) && std::equal(axesB, axesB + n, r.axb.begin())) {
                    plan = r.plan;
                    break;
                }
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (!plan) {
            plan = build_contract_plan(ctx, 1, &A, &B, n, axesA, axesB, compute, &C, nullptr, -1, s);
            if (axes_ok) {
                std::lock_guard<std::mutex> lk(ctx->mu);
                sym_ctx::Recent& r = ctx->recent[static_cast<size_t>(ctx->recent_next)];
                ctx->recent_next = (ctx->recent_next + 1) % static_cast<int>(ctx->recent.size());
                r.a = A->d;
                r.b = B->d;
                r.c = C->d;
                r.n = n;
                r.compute = compute;
                std::copy(axesA, axesA + n, r.axa.begin());
                std::copy(axesB, axesB + n, r.axb.begin());
                r.plan = plan;
            }
        }
        if (!has_data(A) || !has_data(B) || !has_data(C)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        ctx->note(plan);
        run_contract_plan(ctx, *plan, &A, &B, &C, s, true);
    });
}

int32_t sym_contract_noalloc(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n, const int32_t* axesA,
                             const int32_t* axesB, int32_t compute, sym_tensor* C, void* stream) {
    return guard([&] {
        if (!ctx || !A || !B || !C) throw Error(SYM_E_ARG, "NULL argument");
        auto plan = build_noalloc_plan(ctx, A, B, n, axesA, axesB, compute, C);
        if (!has_data(A) || !has_data(B) || !has_data(C)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        run_contract_plan(ctx, *plan, &A, &B, &C, static_cast<hipStream_t>(stream), false);
    });
}

int32_t sym_noalloc_capacity(int64_t* bytes) {
    return guard([&] {
        if (!bytes) throw Error(SYM_E_ARG, "NULL argument");
        *bytes = static_cast<int64_t>(kNoAllocScratchBytes);
    });
}

// ----- backward -----------------------------------------------------------------

int32_t sym_contract_backward(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, const sym_tensor* dC, int32_t n,
                              const int32_t* axesA, const int32_t* axesB, int32_t compute, sym_tensor* dA,
                              sym_tensor* dB, void* stream) {
    return guard([&] {
        if (!ctx || !A || !B || !dC) throw Error(SYM_E_ARG, "NULL argument");
        if (compute != SYM_F32 && compute != SYM_BF16) throw Error(SYM_E_DTYPE, "compute must be F32 or BF16");
        PairInfo p = check_pair(*A->d, *B->d, n, axesA, axesB);
        if (p.su2_general)
            throw Error(SYM_E_UNSUPPORTED, "the backward covers the Abelian groups and the rank-4 SU(2) operator form");
        const Desc& dc = *dC->d;
        if (dA && (dA->d->legs != A->d->legs || dA->d->dtype != SYM_F32 || dA->d->qtot != A->d->qtot || dA->d->tree != A->d->tree))
            throw Error(SYM_E_MISMATCH, "dA does not describe A (FP32)");
        if (dB && (dB->d->legs != B->d->legs || dB->d->dtype != SYM_F32 || dB->d->qtot != B->d->qtot || dB->d->tree != B->d->tree))
            throw Error(SYM_E_MISMATCH, "dB does not describe B (FP32)");
        if (!dA && !dB) return;
        std::ostringstream k;
        k << "B|" << compute << '|' << axes_key(n, axesA, axesB) << '#' << A->d->key << '#' << B->d->key << '#' << dc.key
          << '#' << (dA ? dA->d->key : "-") << '#' << (dB ? dB->d->key : "-");
        std::shared_ptr<BackwardPlan> plan;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            auto it = ctx->backward_plans.find(k.str());
            if (it != ctx->backward_plans.end()) plan = it->second;
        }
        // slots: 0 ws_in, 1 ws_out, 2 A, 3 B, 4 dC, 5 dA, 6 dB
        if (!plan) {
            DescPtr cw = result_desc(*A->d, *B->d, p);
            if (dc.legs != cw->legs || dc.qtot != cw->qtot || dc.group != cw->group || dc.tree != cw->tree)
                throw Error(SYM_E_MISMATCH, "dC does not describe the contraction result");
            plan = std::make_shared<BackwardPlan>();
            plan->gemm.compute = compute;
            for (int i = 0; i < 2; ++i) {
                plan->copy_in[i].src_dtype = i == 0 ? SYM_F32 : SYM_BF16;
                plan->copy_in[i].dst_dtype = compute;
            }
            plan->split.src_dtype = plan->split.dst_dtype = SYM_F32;
            int64_t in_off = 0, out_off = 0;
            auto place_in = [&](const Desc& d) {
                const int64_t b = in_off;
                in_off = align_up(in_off + d.numel, 64);
                return b;
            };
            auto place_out = [&](const Desc& d) {
                const int64_t b = out_off;
                out_off = align_up(out_off + d.numel, 64);
                return b;
            };
            // dC as the M x N operand of dA (K = B's free legs)
            DescPtr dcx = make_desc(cw->group, cw->legs, cw->n_row, cw->tree, cw->qtot, compute, workspace_opts(compute, false));
            // dC^T as the N x M operand of dB (K = A's free legs)
            DescPtr dct = make_desc(cw->group, cw->legs, cw->n_row, cw->tree, cw->qtot, compute, workspace_opts(compute, true));
            const int dc_slot = dc.dtype == SYM_BF16 ? 1 : 0;
            if (dA) {
                DescPtr x = dcx, y = fused_b(*B->d, p, compute, false), z = fused_a(*A->d, p, SYM_F32, false);
                const int64_t xb = place_in(*x), yb = place_in(*y);
                plan->copy_in[dc_slot].add(dc, *x, identity(dc.rank), 4, 0, 0, xb);
                plan->copy_in[B->d->dtype == SYM_BF16 ? 1 : 0].add(*B->d, *y, p.perm_b, 3, 0, 0, yb);
                if (gemm_can_write(*z, *dA->d) && p.perm_a == identity(A->d->rank)) {
                    plan->gemm.add(*dA->d, *x, *y, 5, 0, 0, 0, xb, yb);
                } else {
                    const int64_t zb = place_out(*z);
                    plan->gemm.add(*z, *x, *y, 1, 0, 0, zb, xb, yb);
                    plan->split.add(*z, *dA->d, inverse(p.perm_a), 1, 5, zb, 0);
                }
            }
            if (dB) {
                DescPtr x = fused_a(*A->d, p, compute, true), y = dct, z = fused_b(*B->d, p, SYM_F32, false);
                const int64_t xb = place_in(*x), yb = place_in(*y);
                plan->copy_in[A->d->dtype == SYM_BF16 ? 1 : 0].add(*A->d, *x, p.perm_a, 2, 0, 0, xb);
                plan->copy_in[dc_slot].add(dc, *y, identity(dc.rank), 4, 0, 0, yb);
                if (gemm_can_write(*z, *dB->d) && p.perm_b == identity(B->d->rank)) {
                    plan->gemm.add(*dB->d, *x, *y, 6, 0, 0, 0, xb, yb);
                } else {
                    const int64_t zb = place_out(*z);
                    plan->gemm.add(*z, *x, *y, 1, 0, 0, zb, xb, yb);
                    plan->split.add(*z, *dB->d, inverse(p.perm_b), 1, 6, zb, 0);
                }
            }
            const int var = pick_variant(ctx, compute, k.str());
            plan->grid = ctx->cus() * gemm_blocks_per_cu(compute, var);
            plan->gemm.finalize(var, plan->grid);
            for (auto& c : plan->copy_in) c.finalize();
            plan->split.finalize();
            Allocator alloc = ctx->allocator();
            BuildUploads up;
            if (in_off) plan->ws_in = up.zeroed(alloc, static_cast<size_t>(in_off) * dtype_size(compute));
            if (out_off) plan->ws_out = alloc(static_cast<size_t>(out_off) * sizeof(float));
            for (auto& c : plan->copy_in) c.upload(alloc, &up.copies);
            plan->gemm.upload(alloc, &up.copies);
            plan->split.upload(alloc, &up.copies);
            up.finish(static_cast<hipStream_t>(stream));
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->backward_plans[k.str()] = plan;
        }
        if (!has_data(A) || !has_data(B) || !has_data(dC) || (dA && !has_data(dA)) || (dB && !has_data(dB)))
            throw Error(SYM_E_ARG, "tensor has no data pointer");
        ctx->note(plan);
        PtrTable t{};
        t.p[0] = plan->ws_in ? plan->ws_in->ptr : nullptr;
        t.p[1] = plan->ws_out ? plan->ws_out->ptr : nullptr;
        t.p[2] = A->data;
        t.p[3] = B->data;
        t.p[4] = dC->data;
        t.p[5] = dA ? dA->data : nullptr;
        t.p[6] = dB ? dB->data : nullptr;
        hipStream_t st = static_cast<hipStream_t>(stream);
        for (const auto& c : plan->copy_in) HIP_CHECK(c.launch(t, st));
        HIP_CHECK(plan->gemm.launch(t, plan->grid, st));
        HIP_CHECK(plan->split.launch(t, st));
    });
}

// ----- graphs, timing, tuning ------------------------------------------------------

int32_t sym_graph_create_batched(sym_ctx* ctx, int32_t count, const sym_tensor* const* A, const sym_tensor* const* B,
                                 int32_t n, const int32_t* axesA, const int32_t* axesB, int32_t compute,
                                 sym_tensor* const* C, void* stream, sym_graph** out) {
    return guard([&] {
        if (!ctx || !out || !stream) throw Error(SYM_E_ARG, "ctx, out and a non-null stream are required");
        if (count < 1 || !A || !B || !C) throw Error(SYM_E_ARG, "bad batch");
        hipStream_t s = static_cast<hipStream_t>(stream);
        // chunks of 64 members, as in sym_contract_batched, all captured into
        // one graph; every chunk is checked and planned before the capture
        if (count > 64)
            for (int32_t first = 0; first < count; first += 64)
                (void)contract_key(std::min<int32_t>(64, count - first), A + first, B + first, n, axesA, axesB,
                                   compute, C + first, nullptr);
        auto* g = new sym_graph();
        try {
            for (int32_t first = 0; first < count; first += 64)
                g->plans.push_back(build_contract_plan(ctx, std::min<int32_t>(64, count - first), A + first,
                                                       B + first, n, axesA, axesB, compute, C + first, nullptr, -1,
                                                       s));
        } catch (...) {
            delete g;
            throw;
        }
        if (g->plans.size() == 1 && g->plans[0]->small) {
            try {
                g->table = contract_table(*g->plans[0], A, B, C);
            } catch (...) {
                delete g;
                throw;
            }
            g->direct = true;
            *out = g;
            return;
        }
        try {
            HIP_CHECK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            try {
                for (size_t c = 0; c < g->plans.size(); ++c) {
                    const int32_t first = static_cast<int32_t>(c) * 64;
                    run_contract_plan(ctx, *g->plans[c], A + first, B + first, C + first, s, false);
                }
            } catch (...) {
                hipGraph_t dummy = nullptr;
                (void)hipStreamEndCapture(s, &dummy);
                if (dummy) (void)hipGraphDestroy(dummy);
                throw;
            }
            HIP_CHECK(hipStreamEndCapture(s, &g->graph));
            HIP_CHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        } catch (...) {
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
            if (g->graph) (void)hipGraphDestroy(g->graph);
            delete g;
            throw;
        }
        *out = g;
    });
}

int32_t sym_graph_launch(sym_graph* g, void* stream) {
    return guard([&] {
        if (!g) throw Error(SYM_E_ARG, "graph is NULL");
        if (g->direct) {
            HIP_CHECK(g->plans[0]->small_prog.launch(g->table, static_cast<hipStream_t>(stream)));
            return;
        }
        HIP_CHECK(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    });
}

void sym_graph_destroy(sym_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

int32_t sym_ctx_set_timing(sym_ctx* ctx, int32_t enable) {
    return guard([&] {
        if (!ctx) throw Error(SYM_E_ARG, "ctx is NULL");
        std::lock_guard<std::mutex> lk(ctx->tmu);
        ctx->timing = enable != 0;
    });
}

int32_t sym_ctx_phase_ms(sym_ctx* ctx, int32_t phase, float* ms) {
    return guard([&] {
        if (!ctx || !ms) throw Error(SYM_E_ARG, "NULL argument");
        if (phase < 0 || phase > 2) throw Error(SYM_E_ARG, "phase must be 0, 1 or 2");
        {
            std::lock_guard<std::mutex> lk(ctx->tmu);
            if (!ctx->events_ready) throw Error(SYM_E_ARG, "timing was not enabled for a contraction");
        }
        HIP_CHECK(hipEventElapsedTime(ms, ctx->ev[phase], ctx->ev[phase + 1]));
    });
}

int32_t sym_num_variants(int32_t compute, int32_t* count) {
    return guard([&] {
        if (!count || (compute != SYM_F32 && compute != SYM_BF16)) throw Error(SYM_E_ARG, "bad argument");
        *count = gemm_num_variants(compute);
    });
}

int32_t sym_variant_name(int32_t compute, int32_t variant, const char** name) {
    return guard([&] {
        if (!name || (compute != SYM_F32 && compute != SYM_BF16)) throw Error(SYM_E_ARG, "bad argument");
        if (variant < 0 || variant >= gemm_num_variants(compute)) throw Error(SYM_E_ARG, "no such variant");
        *name = gemm_variant(compute, variant).name;
    });
}

int32_t sym_variant_kernel(int32_t compute, int32_t variant, const char** kernel) {
    return guard([&] {
        if (!kernel || (compute != SYM_F32 && compute != SYM_BF16)) throw Error(SYM_E_ARG, "bad argument");
        if (variant < 0 || variant >= gemm_num_variants(compute)) throw Error(SYM_E_ARG, "no such variant");
        *kernel = gemm_variant_kernel(compute, variant);
    });
}

int32_t sym_default_variant(int32_t compute, int32_t* variant) {
    return guard([&] {
        if (!variant || (compute != SYM_F32 && compute != SYM_BF16)) throw Error(SYM_E_ARG, "bad argument");
        *variant = gemm_default_variant(compute);
    });
}

int32_t sym_ctx_set_variant(sym_ctx* ctx, int32_t compute, int32_t variant) {
    return guard([&] {
        if (!ctx || (compute != SYM_F32 && compute != SYM_BF16)) throw Error(SYM_E_ARG, "bad argument");
        if (variant >= gemm_num_variants(compute)) throw Error(SYM_E_ARG, "no such variant");
        {
            std::lock_guard<std::mutex> lk(ctx->tmu);
            ctx->variant[compute] = variant < 0 ? -1 : variant;
        }
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->forget_recent();
    });
}

int32_t sym_tune_batched(sym_ctx* ctx, int32_t count, const sym_tensor* const* A, const sym_tensor* const* B, int32_t n,
                         const int32_t* axesA, const int32_t* axesB, int32_t compute, sym_tensor* const* C, void* stream,
                         int32_t* best_variant) {
    return guard([&] {
        if (!ctx || !best_variant) throw Error(SYM_E_ARG, "NULL argument");
        if (count > 64) throw Error(SYM_E_UNSUPPORTED, "tuning takes at most 64 contractions");
        hipStream_t s = static_cast<hipStream_t>(stream);
        ctx->ensure_events();
        bool was_timing;
        {
            std::lock_guard<std::mutex> lk(ctx->tmu);
            was_timing = ctx->timing;
            ctx->timing = true;
        }
        std::string key;
        // One host plan for every variant: only the GEMM's tile list depends
        // on the variant, so each candidate is a copy of the plan (sharing its
        // workspaces and device tables) with its own tiles.  The plan runs
        // once; then only GEMM launches are timed.
        auto base = build_contract_plan(ctx, count, A, B, n, axesA, axesB, compute, C, &key, -1, s);
        run_contract_plan(ctx, *base, A, B, C, s, false);
        const PtrTable t = contract_table(*base, A, B, C);
        const int nv = gemm_num_variants(compute);
        std::vector<std::shared_ptr<ContractPlan>> cand(static_cast<size_t>(nv));
        Allocator alloc = ctx->allocator();
        // With at least eight tiles of the default variant per CU there is
        // parallelism enough for the large tiles, and tiles of a quarter of
        // their area or less only re-read the operands more often (on the
        // 64-member batch the 128 x 128 and 64 x 64 kernels ran 2.8 and 5.5
        // times slower): those are not timed.
        const GemmVariant dv = gemm_variant(compute, gemm_default_variant(compute));
        const bool big = static_cast<int64_t>(base->gemm.tiles.size()) >= 8LL * ctx->cus();
        auto skipped = [&](int v) {
            const GemmVariant gv = gemm_variant(compute, v);
            return big && 4LL * gv.mt * gv.nt <= static_cast<int64_t>(dv.mt) * dv.nt;
        };
        for (int v = 0; v < nv; ++v) {
            if (skipped(v)) continue;
            auto c = std::make_shared<ContractPlan>(*base);
            c->requested_variant = v;
            c->grid = ctx->cus() * gemm_blocks_per_cu(compute, v);
            c->gemm.finalize(v, c->grid);
            BuildUploads up;
            c->gemm.d_tiles = upload_table(alloc, c->gemm.tiles, &up.copies);
            up.finish(s);
            cand[static_cast<size_t>(v)] = c;
        }
        // in the second pass each timed GEMM launch follows the plan's fuse
        // (its time not counted), so that it meets the caches and the clock
        // the way it does in the call it serves
        auto time_gemm = [&](const ContractPlan& c, bool after_fuse) {
            if (after_fuse) {
                for (const auto& f : base->fuse) HIP_CHECK(f.launch(t, s));
                for (const auto& r : base->rc_pre) HIP_CHECK(r.prog.launch(t, r.in_slot, r.out_slot, s));
            }
            HIP_CHECK(hipEventRecord(ctx->ev[1], s));
            HIP_CHECK(c.gemm.launch(t, c.grid, s));
            HIP_CHECK(hipEventRecord(ctx->ev[2], s));
            HIP_CHECK(hipStreamSynchronize(s));
            float ms = 0.f;
            HIP_CHECK(hipEventElapsedTime(&ms, ctx->ev[1], ctx->ev[2]));
            return ms;
        };
        // first pass: one launch each; second pass: three more for the (at
        // most five) fastest variants within 8 % of the fastest and the
        // default, taken round-robin so that a drift of the clock (power and
        // thermal state) weighs on every candidate alike.  The smallest sum
        // of second-pass times wins, unless the default variant is within
        // 1 % of it: the default then stays.
        std::vector<float> first(static_cast<size_t>(nv));
        float fastest = -1.f;
        for (int v = 0; v < nv; ++v) {
            if (!cand[static_cast<size_t>(v)]) continue;
            first[static_cast<size_t>(v)] = time_gemm(*cand[static_cast<size_t>(v)], false);
            if (fastest < 0.f || first[static_cast<size_t>(v)] < fastest) fastest = first[static_cast<size_t>(v)];
        }
        std::vector<int> keep;
        for (int v = 0; v < nv; ++v)
            if (cand[static_cast<size_t>(v)] && first[static_cast<size_t>(v)] <= 1.08f * fastest) keep.push_back(v);
        std::stable_sort(keep.begin(), keep.end(), [&](int x, int y) {
            return first[static_cast<size_t>(x)] < first[static_cast<size_t>(y)];
        });
        if (keep.size() > 5) keep.resize(5);
        const int def = gemm_default_variant(compute);
        if (std::find(keep.begin(), keep.end(), def) == keep.end()) keep.push_back(def);
        std::vector<float> total(static_cast<size_t>(nv), 0.f);
        for (int rep = 0; rep < 3; ++rep)
            for (int v : keep) total[static_cast<size_t>(v)] += time_gemm(*cand[static_cast<size_t>(v)], true);
        int best = keep[0];
        for (int v : keep)
            if (total[static_cast<size_t>(v)] < total[static_cast<size_t>(best)]) best = v;
        if (total[static_cast<size_t>(def)] <= 1.01f * total[static_cast<size_t>(best)]) best = def;
        const std::string tk = std::to_string(compute) + ":" + std::to_string(std::hash<std::string>{}(key));
        {
            std::lock_guard<std::mutex> lk(ctx->tmu);
            ctx->timing = was_timing;
            ctx->tuned[tk] = best;
        }
        {
            // the winner becomes the cached plan of the structure
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->contract_plans[key] = cand[static_cast<size_t>(best)];
            ctx->forget_recent();
        }
        if (const char* f = std::getenv("SYM_TUNE_CACHE")) {
            std::ofstream o(f, std::ios::app);
            o << tk << ' ' << best << '\n';
        }
        *best_variant = best;
    });
}

// ----- block-wise SVD -------------------------------------------------------

namespace {

// eig: the eigen-decomposition of each sector's symmetric part, which needs
// square sector matrices
std::shared_ptr<SvdPlan> svd_plan_of(const Desc& d, bool eig) {
    auto plan = std::make_shared<SvdPlan>();
    if (d.opts.trans) throw Error(SYM_E_UNSUPPORTED, "transposed layouts have no SVD");
    for (const Sector& sc : d.sectors) {
        if (sc.rows == 0 || sc.cols == 0) continue;
        if (eig && sc.rows != sc.cols) throw Error(SYM_E_UNSUPPORTED, "eigen-decomposition needs square sector matrices");
        SvdProb p{};
        p.sym = eig ? 1 : 0;
        p.M = static_cast<int32_t>(sc.rows);
        p.N = static_cast<int32_t>(sc.cols);
        p.ld = static_cast<int32_t>(sc.ld);
        p.k = std::min(p.M, p.N);
        p.L = std::max(p.M, p.N);
        if (p.k > kSvdMaxK) throw Error(SYM_E_UNSUPPORTED, "sector with min(rows, cols) above 4096");
        p.rows_are_vectors = p.M <= p.N ? 1 : 0;
        p.src_off = sc.offset;
        p.w_off = plan->w_elems;
        p.q_off = plan->q_elems;
        p.u_off = plan->u_elems;
        p.s_off = plan->s_elems;
        p.vt_off = plan->vt_elems;
        plan->w_elems += static_cast<int64_t>(p.k) * p.L;
        plan->q_elems += static_cast<int64_t>(p.k) * p.k;
        plan->u_elems += static_cast<int64_t>(p.M) * p.k;
        plan->s_elems += p.k;
        plan->vt_elems += static_cast<int64_t>(p.k) * p.N;
        plan->probs.push_back(p);
    }
    plan->pair_start.push_back(0);
    for (const SvdProb& p : plan->probs) {
        // block pairs of the block-Jacobi rounds: blocks of kSvdBlock vectors,
        // their count rounded up to even
        const int32_t nb = (p.k + kSvdBlock - 1) / kSvdBlock, nbp = nb + (nb & 1);
        plan->pair_start.push_back(plan->pair_start.back() + nbp / 2);
        plan->max_kp = std::max(plan->max_kp, nbp);
    }
    return plan;
}

// W = U Vt (M x N) and P = V diag(S) Vt (rows >= columns) or U diag(S) U^T
// (k x k) of every sector, with U at offset 0 and Vt at offset u_elems of
// one buffer
void polar_tables(SvdPlan& plan) {
    std::vector<PolarGemm> wp, pp;
    for (const SvdProb& p : plan.probs) {
        const int64_t vt0 = plan.u_elems + p.vt_off;
        PolarGemm w{};
        w.a_off = p.u_off;
        w.as0 = p.k;
        w.as1 = 1;
        w.b_off = vt0;
        w.bs0 = p.N;
        w.bs1 = 1;
        w.m = p.M;
        w.n = p.N;
        w.kk = p.k;
        w.d_off = -1;
        w.c_off = plan.pw_elems;
        w.ldc = p.N;
        w.which = 0;
        plan.pw_elems += static_cast<int64_t>(p.M) * p.N;
        wp.push_back(w);
        PolarGemm q{};
        if (p.M >= p.N) {   // V diag(S) Vt: A(i, l) = Vt[l][i], B(l, j) = Vt[l][j]
            q.a_off = vt0;
            q.as0 = 1;
            q.as1 = p.N;
            q.b_off = vt0;
            q.bs0 = p.N;
            q.bs1 = 1;
        } else {            // U diag(S) U^T: A(i, l) = U[i][l], B(l, j) = U[j][l]
            q.a_off = p.u_off;
            q.as0 = p.k;
            q.as1 = 1;
            q.b_off = p.u_off;
            q.bs0 = 1;
            q.bs1 = p.k;
        }
        q.m = q.n = q.kk = p.k;
        q.d_off = p.s_off;
        q.c_off = plan.pp_elems;
        q.ldc = p.k;
        q.which = 1;
        plan.pp_elems += static_cast<int64_t>(p.k) * p.k;
        pp.push_back(q);
    }
    plan.pgemm = wp;
    plan.pgemm.insert(plan.pgemm.end(), pp.begin(), pp.end());
    for (size_t g = 0; g < plan.pgemm.size(); ++g) {
        const PolarGemm& q = plan.pgemm[g];
        for (int32_t i0 = 0; i0 < q.m; i0 += kPolarTile)
            for (int32_t j0 = 0; j0 < q.n; j0 += kPolarTile) plan.ptiles.push_back({static_cast<int32_t>(g), i0, j0, 0});
        if (g + 1 == wp.size()) plan.n_wtiles = static_cast<int32_t>(plan.ptiles.size());
    }
}

}  // namespace

int32_t sym_svd_sizes(const sym_tensor* T, int64_t* u_elems, int64_t* s_elems, int64_t* vt_elems) {
    return guard([&] {
        if (!T || !u_elems || !s_elems || !vt_elems) throw Error(SYM_E_ARG, "NULL argument");
        auto plan = svd_plan_of(*T->d, false);
        *u_elems = plan->u_elems;
        *s_elems = plan->s_elems;
        *vt_elems = plan->vt_elems;
    });
}

namespace {

// the cached plan of T's structure (one per mode), built and uploaded on the
// first call
std::shared_ptr<SvdPlan> svd_plan_cached(sym_ctx* ctx, const sym_tensor* T, bool eig, hipStream_t stream,
                                         bool polar = false) {
    const std::string key = (eig ? "E|" : polar ? "P|" : "S|") + T->d->key;
    std::shared_ptr<SvdPlan> plan;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->svd_plans.find(key);
        if (it != ctx->svd_plans.end()) plan = it->second;
    }
    if (plan) return plan;
    plan = svd_plan_of(*T->d, eig);
    Allocator alloc = ctx->allocator();
    if (!plan->probs.empty()) {
        BuildUploads up;
        plan->d_probs = alloc(plan->probs.size() * sizeof(SvdProb));
        up.copies.push_back({plan->d_probs->ptr, plan->probs.data(), plan->probs.size() * sizeof(SvdProb)});
        plan->d_pairs = alloc(plan->pair_start.size() * sizeof(int32_t));
        up.copies.push_back({plan->d_pairs->ptr, plan->pair_start.data(), plan->pair_start.size() * sizeof(int32_t)});
        up.finish(stream);
        plan->w = alloc(static_cast<size_t>(plan->w_elems) * sizeof(double));
        plan->q = alloc(static_cast<size_t>(plan->q_elems) * sizeof(double));
        plan->flag = alloc(sizeof(int32_t));
        plan->lastrot = alloc(static_cast<size_t>(std::max<int32_t>(1, 2 * plan->pair_start.back())) * sizeof(int32_t));
        plan->scale = alloc(plan->probs.size() * sizeof(double));
        if (eig) plan->shift = alloc(plan->probs.size() * sizeof(double));
        if (polar) {
            polar_tables(*plan);
            plan->uv = alloc(static_cast<size_t>(plan->u_elems + plan->vt_elems) * sizeof(double));
            plan->s = alloc(static_cast<size_t>(plan->s_elems) * sizeof(double));
            BuildUploads pu;
            plan->d_pgemm = alloc(plan->pgemm.size() * sizeof(PolarGemm));
            pu.copies.push_back({plan->d_pgemm->ptr, plan->pgemm.data(), plan->pgemm.size() * sizeof(PolarGemm)});
            plan->d_ptiles = alloc(plan->ptiles.size() * sizeof(PolarTile));
            pu.copies.push_back({plan->d_ptiles->ptr, plan->ptiles.data(), plan->ptiles.size() * sizeof(PolarTile)});
            pu.finish(stream);
        }
        plan->gpart = alloc(static_cast<size_t>(std::max<int32_t>(1, plan->pair_start.back())) * kSvdSlices *
                            (4 * kSvdBlock * kSvdBlock) * sizeof(double));
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->svd_plans[key] = plan;
    return plan;
}

void run_svd(const sym_tensor* T, SvdPlan& plan, double* U, double* S, double* Vt, int32_t* sweeps, int32_t max_sweeps,
             hipStream_t stream) {
    int32_t done = 0;
    HIP_CHECK(launch_svd(T->d->dtype, T->data, static_cast<const SvdProb*>(plan.d_probs->ptr),
                         static_cast<const int32_t*>(plan.d_pairs->ptr), static_cast<int32_t>(plan.probs.size()),
                         plan.pair_start.back(), plan.max_kp, static_cast<double*>(plan.w->ptr),
                         static_cast<double*>(plan.q->ptr), U, S, Vt, static_cast<double*>(plan.scale->ptr),
                         plan.shift ? static_cast<double*>(plan.shift->ptr) : nullptr,
                         static_cast<double*>(plan.gpart->ptr), static_cast<int32_t*>(plan.lastrot->ptr),
                         static_cast<int32_t*>(plan.flag->ptr),
                         &plan.flag_host, max_sweeps, &done, stream));
    if (sweeps) *sweeps = done;
}

}  // namespace

int32_t sym_svd(sym_ctx* ctx, const sym_tensor* T, double* U, double* S, double* Vt, int32_t* sweeps,
                int32_t max_sweeps, void* stream) {
    // one plan per structure; calls with the same structure on one context
    // share its workspaces, so they must not overlap in time
    return guard([&] {
        if (!ctx || !T) throw Error(SYM_E_ARG, "NULL argument");
        if (!has_data(T)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        if (max_sweeps < 1) throw Error(SYM_E_ARG, "max_sweeps must be >= 1");
        auto plan = svd_plan_cached(ctx, T, false, static_cast<hipStream_t>(stream));
        if (sweeps) *sweeps = 0;
        if (plan->probs.empty()) return;   // no sector: nothing to factorise or write
        if (!U || !S || !Vt) throw Error(SYM_E_ARG, "NULL argument");
        ctx->note(plan);
        run_svd(T, *plan, U, S, Vt, sweeps, max_sweeps, static_cast<hipStream_t>(stream));
    });
}

int32_t sym_eigh_sizes(const sym_tensor* T, int64_t* v_elems, int64_t* w_elems) {
    return guard([&] {
        if (!T || !v_elems || !w_elems) throw Error(SYM_E_ARG, "NULL argument");
        auto plan = svd_plan_of(*T->d, true);
        *v_elems = plan->u_elems;
        *w_elems = plan->s_elems;
    });
}

int32_t sym_eigh(sym_ctx* ctx, const sym_tensor* T, double* V, double* w, int32_t* sweeps, int32_t max_sweeps,
                 void* stream) {
    return guard([&] {
        if (!ctx || !T) throw Error(SYM_E_ARG, "NULL argument");
        if (!has_data(T)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        if (max_sweeps < 1) throw Error(SYM_E_ARG, "max_sweeps must be >= 1");
        auto plan = svd_plan_cached(ctx, T, true, static_cast<hipStream_t>(stream));
        if (sweeps) *sweeps = 0;
        if (plan->probs.empty()) return;
        if (!V || !w) throw Error(SYM_E_ARG, "NULL argument");
        ctx->note(plan);
        run_svd(T, *plan, V, w, nullptr, sweeps, max_sweeps, static_cast<hipStream_t>(stream));
    });
}

int32_t sym_polar_sizes(const sym_tensor* T, int64_t* w_elems, int64_t* p_elems) {
    return guard([&] {
        if (!T || !w_elems || !p_elems) throw Error(SYM_E_ARG, "NULL argument");
        auto plan = svd_plan_of(*T->d, false);
        polar_tables(*plan);
        *w_elems = plan->pw_elems;
        *p_elems = plan->pp_elems;
    });
}

int32_t sym_polar(sym_ctx* ctx, const sym_tensor* T, double* W, double* P, int32_t* sweeps, int32_t max_sweeps,
                  void* stream) {
    return guard([&] {
        if (!ctx || !T) throw Error(SYM_E_ARG, "NULL argument");
        if (!has_data(T)) throw Error(SYM_E_ARG, "tensor has no data pointer");
        if (max_sweeps < 1) throw Error(SYM_E_ARG, "max_sweeps must be >= 1");
        auto plan = svd_plan_cached(ctx, T, false, static_cast<hipStream_t>(stream), true);
        if (sweeps) *sweeps = 0;
        if (plan->probs.empty()) return;
        if (!W) throw Error(SYM_E_ARG, "NULL argument");
        ctx->note(plan);
        double* uv = static_cast<double*>(plan->uv->ptr);
        double* sv = static_cast<double*>(plan->s->ptr);
        run_svd(T, *plan, uv, sv, uv + plan->u_elems, sweeps, max_sweeps, static_cast<hipStream_t>(stream));
        // the W products always; the P products only when P is wanted
        const int32_t n = P ? static_cast<int32_t>(plan->ptiles.size()) : plan->n_wtiles;
        HIP_CHECK(launch_polar(static_cast<const PolarGemm*>(plan->d_pgemm->ptr),
                               static_cast<const PolarTile*>(plan->d_ptiles->ptr), n, uv, sv, W, P,
                               static_cast<hipStream_t>(stream)));
    });
}

int32_t sym_svd_truncate(const sym_tensor* T, const double* S, int64_t chi_max, double tol, int32_t* keep,
                         double* discarded) {
    return guard([&] {
        if (!T || !S || !keep) throw Error(SYM_E_ARG, "NULL argument");
        if (chi_max < 0) throw Error(SYM_E_ARG, "chi_max must be >= 0");
        auto plan = svd_plan_of(*T->d, false);
        // (value, weight, sector) over every singular value; an SU(2) sector
        // of coupled spin e (label 2e) stands for 2e + 1 equal values
        struct Item { double v; int32_t w; int32_t s; };
        std::vector<Item> items;
        std::vector<int32_t> weight;
        size_t pi = 0;
        for (size_t si = 0; si < T->d->sectors.size(); ++si) {
            const Sector& sc = T->d->sectors[si];
            keep[si] = 0;
            if (sc.rows == 0 || sc.cols == 0) continue;
            const SvdProb& p = plan->probs[pi++];
            const int32_t w = T->d->group == SYM_SU2 ? sc.label + 1 : 1;
            for (int32_t j = 0; j < p.k; ++j) items.push_back({S[p.s_off + j], w, static_cast<int32_t>(si)});
        }
        std::stable_sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.v > b.v; });
        int64_t used = 0;
        double lost = 0.0;
        bool open = true;
        for (const Item& it : items) {
            if (open && it.v > tol && used + it.w <= chi_max) {
                used += it.w;
                ++keep[it.s];
            } else {
                open = false;   // keep exactly the largest values: stop at the first that does not fit
                lost += it.w * it.v * it.v;
            }
        }
        if (discarded) *discarded = lost;
    });
}

double sym_fmove_coeff(int32_t tjA, int32_t tjB, int32_t tjC, int32_t tjJ, int32_t tjD, int32_t tjE) {
    double v = std::numeric_limits<double>::quiet_NaN();
    (void)guard([&] { v = fmove_coeff(tjA, tjB, tjC, tjJ, tjD, tjE); });
    return v;
}

}  // extern "C"
