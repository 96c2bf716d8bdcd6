/*
 * symtensor: contraction of U(1)- and SU(2)-symmetric tensors stored as
 * charge-sector blocks, on AMD Instinct MI355X (gfx950).
 *
 * Terms follow the thesis (Singh, "Tensor Network States and Algorithms in the
 * presence of Abelian and non-Abelian Symmetries", arXiv:1203.2222):
 *
 *  - A tensor is a multidimensional array whose indices ("legs") each carry a
 *    direction, in or out (section "Tensors as linear maps").
 *  - A symmetric tensor is stored by its degeneracy tensors ("blocks"): one
 *    dense block per allowed tuple of leg labels, plus, for SU(2), one per
 *    intermediate spin of its fusion tree (section "Block structure of
 *    SU(2)-invariant tensors", eq:datak).  The structural tensors are never
 *    stored.
 *  - A leg is described by its spectrum: labels with their degeneracies
 *    (eq:decoV).  For U(1) a label is a charge q; for SU(2) it is twice the
 *    spin, 2j.  Labels are strictly ascending.
 *  - U(1) charge rule: a block is allowed when sum(q, out legs) minus
 *    sum(q, in legs) equals the tensor's total charge (0 for an invariant
 *    tensor).  This is the invariance condition eq:Tinv with exp(i r q) on
 *    every leg.
 *  - SU(2) tensors of rank 4 may use one of three trees (eq:cob1, eq:cob2,
 *    eq:deco41): OPERATOR (in,in,out,out), (1,2)->e->(3,4); LEFT
 *    (in,in,in,out), {1,2->e; e,3->4}; RIGHT (in,in,in,out), {2,3->f; 1,f->4}.
 *    SU(2) tensors of any rank (1..8) and any arrows use the CHAIN tree (a
 *    tree decomposition, eq:datastruct, with left-associative fusion trees):
 *    the incoming legs, in leg order c_0, c_1, .., are fused as
 *    (c_0, c_1 -> a_1), (a_1, c_2 -> a_2), .. to a total spin J, the outgoing
 *    legs d_0, d_1, .. likewise (b_1, b_2, ..) to the same J (an empty chain
 *    has total 0).  A block is a label tuple with its free intermediate
 *    spins (a_1 .. a_{n-2}, J when both chains have two legs or more,
 *    b_1 .. b_{m-2}), blocks of one label tuple ordered by that key.  With
 *    arrows (in,in,out,out) it is the OPERATOR tree, with (in,in,in,out) the
 *    LEFT tree, with the same blocks.
 *    Every node obeys the fusion rule eq:fusionrules.
 *
 * Data layout ("sector-major for a bipartition").  A tensor declares n_row:
 * its first n_row legs are row legs, the rest column legs.  Its data is one
 * row-major matrix per sector, packed back to back in ascending sector order
 * with no padding:
 *  - U(1): the sector of a row-label tuple is the charge flowing in through
 *    the row legs, s = sum(q, in row legs) - sum(q, out row legs); a column
 *    tuple belongs to s = sum(q, out col legs) - sum(q, in col legs) - qtot.
 *  - SU(2) (n_row = 2, OPERATOR or LEFT tree): the sector is the intermediate
 *    spin e; a row pair (j1,j2) appears in every sector e it can fuse to.
 *  - SU(2) CHAIN tree (0 < n_row < rank, the first n_row legs incoming): the
 *    sector is the coupled spin a_{n_row-1} of the row legs; a row tuple is
 *    the row labels with a_1 .. a_{n_row-2}, a column tuple the other labels
 *    with the remaining intermediate spins; tuples are ordered labels first,
 *    then spins.
 *  - Inside a sector, rows run over row-label tuples in lexicographic order,
 *    each spanning the row-major product of its row-leg degeneracies; columns
 *    likewise over column-label tuples.  This is the fuse of eq:fuse with the
 *    last index fastest.
 * With n_row = 0 or n_row = rank there is a single sector and the data is the
 * canonical block list: blocks in lexicographic order of their label tuple
 * (SU(2): intermediate spin last), each block row-major, back to back.
 *
 * Contraction (eq:tensormult, the five steps eq:multi1-eq:multi5, and the
 * block-wise multiply eq:blockmult): C = A . B over A's legs axesA[i] paired
 * with B's legs axesB[i].  Paired legs must carry identical spectra and
 * opposite arrows.  C's legs are A's free legs (in order) then B's free legs;
 * C has n_row = number of A's free legs and qtot = qtot(A) + qtot(B).
 * Internally each operand is fused (permute + reshape) into per-sector
 * matrices, one GEMM runs per sector, and the product is split into C.
 *
 * Memory.  Tensor handles describe data they do not own: the caller passes a
 * device pointer (torch storage in the Python binding) and keeps it alive.
 * The library allocates its own workspaces through the context's allocator
 * callback (hipMalloc when none is given) and keeps them with the cached plan.
 *
 * Errors.  Every call returns a status; nothing throws across the ABI.  All
 * validation happens on the host before any launch, so a failed call leaves
 * outputs untouched.  sym_last_error() returns a thread-local message.
 *
 * Streams.  Kernels are launched on the hipStream_t passed as `stream` (NULL =
 * the null stream).  The library never synchronises a stream except in
 * sym_graph_create_batched, sym_svd and the first call on a new structure
 * (which builds its plan).
 *
 * Overlapping calls.  A plan is cached per structure (the tensors' leg
 * descriptions, the axes and the compute type) and owns that structure's
 * workspaces.  Calls that use the same plan (sym_contract, sym_contract_batched,
 * sym_contract_backward, sym_svd on equal structures, and replays of a graph
 * built from that plan) write the same workspaces: they must not run at the
 * same time, whether on different streams, from different threads, or beside
 * a graph replay.  Calls on different structures, or on different contexts,
 * may overlap.
 */
#ifndef SYMTENSOR_H
#define SYMTENSOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SYM_OK = 0,
    SYM_E_ARG = 1,          /* null pointer, bad rank, bad axes or permutation      */
    SYM_E_SPECTRUM = 2,     /* contracted legs carry different spectra              */
    SYM_E_ARROW = 3,        /* contracted legs with the same arrow; SU(2) tree arrows */
    SYM_E_CHARGE = 4,       /* labels not strictly ascending, negative 2j           */
    SYM_E_DTYPE = 5,        /* unsupported data type combination                    */
    SYM_E_NOMEM = 6,        /* allocator returned NULL                               */
    SYM_E_HIP = 7,          /* a HIP runtime call failed                             */
    SYM_E_UNSUPPORTED = 8,  /* valid request outside what this library implements    */
    SYM_E_MISMATCH = 9      /* output handle does not describe the expected result  */
};

/* Groups.  Abelian ones (section "Conclusions and outlook": fusion rules of
 * composite groups and of fermion parity) use one int32 label per irrep:
 *   SYM_U1   charge q; a block is allowed when sum_out q - sum_in q = qtot.
 *   SYM_Z2   parity p in {0, 1}; the same rule modulo 2 (qtot in {0, 1}).
 *   SYM_U1U1 a pair (q1, q2) with -2048 <= q1, q2 < 2048, stored as
 *            q1 * 65536 + q2 (label order is then (q1, q2) lexicographic);
 *            the U(1) rule holds for each component (qtot stored the same way).
 *   SYM_Z2F  fermion parity: the Z2 rule, and every permutation of legs
 *            multiplies a block by the swap factor R(1,1->0) = -1 once for
 *            each pair of odd legs whose order it reverses (R = 1 otherwise,
 *            F = 1); a contraction moves A's contracted legs behind its free
 *            legs and B's in front of its own, in the order axesA / axesB
 *            give, then multiplies.
 *   SYM_SU2  doubled spin 2j >= 0 on rank-4 trees (see sym_tensor_create). */
enum { SYM_U1 = 0, SYM_SU2 = 1, SYM_Z2 = 2, SYM_U1U1 = 3, SYM_Z2F = 4 };   /* group */
enum { SYM_F32 = 0, SYM_BF16 = 1 };                /* element type                */
enum { SYM_IN = 0, SYM_OUT = 1 };                  /* leg direction               */
enum { SYM_TREE_NONE = 0, SYM_TREE_OPERATOR = 1,   /* SU(2) coupling tree         */
       SYM_TREE_LEFT = 2, SYM_TREE_RIGHT = 3, SYM_TREE_CHAIN = 4 };

#define SYM_MAX_RANK 8

/* One leg: n labels (ascending), their degeneracies (>= 1) and the arrow.
 * The arrays are copied by sym_tensor_create. */
typedef struct {
    int32_t n;
    const int32_t* label;   /* see the group list: q, p, encoded (q1, q2), or 2j */
    const int64_t* deg;
    int32_t arrow;          /* SYM_IN or SYM_OUT */
} sym_leg;

typedef struct sym_ctx sym_ctx;
typedef struct sym_tensor sym_tensor;
typedef struct sym_graph sym_graph;

typedef void* (*sym_alloc_fn)(size_t bytes, void* user);
typedef void (*sym_free_fn)(void* ptr, void* user);

/* Context: allocator bridge and plan cache.  alloc/free may be NULL (then
 * hipMalloc/hipFree).  Creating a context touches no GPU.  Plan caches are
 * guarded by a lock, so one context may be used from several threads (subject
 * to the overlap rule above).
 * Plans are built on the first call with a new structure: their device
 * tables are copied, and their fused-operand workspaces cleared, on that
 * call's stream, and the call then waits for that stream (never for the whole
 * device) before it caches the plan, which is from then on ready for calls
 * on any stream.  Memory alloc returns during such a call must therefore be
 * free for use in the order of the call's stream (a stream-ordered pool for
 * that stream, or memory with no pending work). */
int32_t sym_ctx_create(sym_alloc_fn alloc, sym_free_fn free_fn, void* user, sym_ctx** out);
void sym_ctx_destroy(sym_ctx* ctx);
/* Drop every cached plan; a plan's workspaces are freed when nothing else
 * (a sym_graph, a sym_hold) still refers to it. */
int32_t sym_ctx_clear(sym_ctx* ctx);

/* Holds: keep plans alive for a graph captured outside the library (the
 * thesis' "precompute once, reuse every iteration" structure replayed from a
 * captured iteration).  Between sym_hold_begin and sym_hold_end every plan a
 * compute call on ctx uses (contraction, backward, permute, recoupling, SVD)
 * is added to the hold, and stays allocated, device tables and workspaces
 * included, until sym_hold_destroy, whatever happens to the context's caches
 * meanwhile (sym_ctx_clear, sym_tune_batched, a plan rebuilt for another tile
 * variant).  One hold collects at a time per context (SYM_E_ARG otherwise).
 * sym_hold_count gives the number of plans held.  Destroying a hold frees
 * nothing the caches still use; a hold must be destroyed while the
 * context's allocator callbacks can still be called.  Pure host work. */
typedef struct sym_hold sym_hold;
int32_t sym_hold_begin(sym_ctx* ctx, sym_hold** out);
int32_t sym_hold_end(sym_ctx* ctx);
int32_t sym_hold_count(const sym_hold* h, int64_t* n);
void sym_hold_destroy(sym_hold* h);

/* Describe a symmetric tensor (section "Block structure"; eq:datak).
 * group: one of the groups above; rank <= SYM_MAX_RANK (SU(2) rank-4 trees:
 * 4); n_row in [0, rank] (rank-4 SU(2) trees: 0, 2 or 4, and 2 only on the
 * OPERATOR or LEFT tree; CHAIN: 0 or rank, or a bipartition whose row legs
 * are incoming); tree: SU(2) tree id (SYM_TREE_NONE for the Abelian groups);
 * qtot: total charge of
 * an Abelian tensor (0 = invariant; must be 0 for SU(2)); dtype: SYM_F32 or
 * SYM_BF16; data: device pointer to
 * numel elements in the layout described above, borrowed (may be NULL and set
 * later with sym_tensor_set_data).  Compute calls fail with SYM_E_ARG on a
 * tensor whose buffer is still NULL, unless numel is 0 (no allowed block:
 * nothing is read or written).  Pure host work. */
int32_t sym_tensor_create(sym_ctx* ctx, int32_t group, int32_t rank, const sym_leg* legs,
                          int32_t n_row, int32_t tree, int32_t qtot, int32_t dtype,
                          void* data, sym_tensor** out);
void sym_tensor_destroy(sym_tensor* t);
int32_t sym_tensor_set_data(sym_tensor* t, void* data);
int32_t sym_tensor_numel(const sym_tensor* t, int64_t* numel);
int32_t sym_tensor_num_blocks(const sym_tensor* t, int64_t* n_blocks);
int32_t sym_tensor_num_sectors(const sym_tensor* t, int64_t* n_sectors);
/* Block i in canonical order: its labels[rank], intermediate spin (-1 for
 * U(1)), element offset of its first entry in the data, shape[rank] and the
 * element stride of each leg inside the data (any output may be NULL). */
int32_t sym_tensor_block_info(const sym_tensor* t, int64_t i, int32_t* labels, int32_t* internal,
                              int64_t* offset, int64_t* shape, int64_t* strides);
/* SU(2) CHAIN tree: the free intermediate spins (doubled) of block i, its
 * key within its label tuple: (a_1 .. a_{n-2}, J when both chains have two
 * legs or more, b_1 .. b_{m-2}) (see sym_tensor_create); *n_inner receives
 * their number (0 for other trees and groups); inner may be NULL. */
int32_t sym_tensor_block_inner(const sym_tensor* t, int64_t i, int32_t* inner, int32_t* n_inner);
/* Sector i: its label (U(1) charge or SU(2) 2e), rows, cols, element offset. */
int32_t sym_tensor_sector_info(const sym_tensor* t, int64_t i, int32_t* label, int64_t* rows,
                               int64_t* cols, int64_t* offset);

/* PERMUTE + FUSE (eq:permute, eq:fuse, eq:split; chapter "Implementation of
 * non-Abelian symmetries II", PERMUTE).  out's legs are in's legs reordered as
 * out.leg[i] = in.leg[perm[i]], with n_row_out row legs and element type
 * dtype_out (F32->BF16 rounds to nearest even).
 *  - U(1): any permutation and bipartition; a pure block gather.
 *  - SU(2): perm = identity changes only the layout; perm = (0,2,1,3) on a
 *    LEFT-tree tensor recouples it to the RIGHT tree on legs (1,3,2,4) by the
 *    F-move (eq:fmove2, F from 6j symbols by Racah's formula, FP64) followed
 *    by the swap of legs 2 and 3 with phase (-1)^(j2+j3-f) (eq:perm11); the
 *    output then has n_row_out = 0 or 4 (canonical block list).
 * sym_permute_fuse_output creates the handle of the result (data may be
 * NULL).  sym_permute_fuse writes into out, which must describe that result,
 * in the packed layout or in a contraction's operand layout
 * (sym_contract_operand_output: the same legs, rows and element type, padded
 * and possibly transposed sector matrices, whose padding it leaves as it
 * is); in and out must not overlap. */
int32_t sym_permute_fuse_output(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm,
                                int32_t n_row_out, int32_t dtype_out, void* data, sym_tensor** out);
int32_t sym_permute_fuse(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t n_row_out,
                         sym_tensor* out, void* stream);

/* General SU(2) PERMUTE of a rank-4 tensor to a chosen tree (the routine
 * PERMUTE with the matrix Gamma(tree, p, tree') of eq:permsu2 and eq:Gamma),
 * combined with REVERSE (section "Reversal of indices") of every leg whose
 * arrow the target tree changes.  out's leg i is in's leg perm[i] with the
 * same spectrum and the arrow of slot i of tree_out (OPERATOR
 * (in,in,out,out), LEFT or RIGHT (in,in,in,out)); any permutation and any of
 * the three trees is accepted.  For each label tuple the output blocks are
 * y_f = sum_e Gamma[f][e] x_e (legs permuted), Gamma composed on the host in
 * FP64 from F-moves (eq:fmove2, 6j by Racah's formula), swap factors
 * (-1)^(ja+jb-jc) (eq:braid3) and, per reversed leg, the bend factor
 * sqrt((2e+1)/(2j4+1)) or its inverse; the combination runs on the device in
 * FP64 on FP32 data.  Reversal convention: an outgoing leg is reversed by the
 * cup (eq:cupj) and an incoming one by the cap (eq:capj), the leg's m index
 * summed against the matrix's row index.
 * in: SU(2), FP32, any layout; n_row_out: 0 or 4, or 2 when tree_out is
 * OPERATOR or LEFT.  SYM_E_UNSUPPORTED for Abelian tensors (use
 * sym_permute_fuse).  sym_permute_tree_output creates the result's handle
 * (data may be NULL); sym_permute_tree writes into out, which must describe
 * exactly that result; in and out must not overlap.  The plan (Gamma of
 * every label tuple) is built on the first call and cached. */
int32_t sym_permute_tree_output(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t tree_out,
                                int32_t n_row_out, void* data, sym_tensor** out);
int32_t sym_permute_tree(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, int32_t tree_out,
                         int32_t n_row_out, sym_tensor* out, void* stream);
/* General SU(2) PERMUTE with REVERSE onto the CHAIN tree, at any rank (the
 * routine PERMUTE with Gamma(tree, p, tree') of eq:permsu2 and eq:Gamma,
 * section "Tree decompositions of SU(2)-invariant tensors", and REVERSE of
 * section "Reversal of indices").  out's leg i is in's leg perm[i] (same
 * spectrum) with arrow arrows_out[i]; every leg whose arrow changes is
 * reversed (an outgoing leg by the cup of eq:cupj, an incoming one by the cap
 * of eq:capj, the leg's m index summed against the matrix's row index).  For
 * each label tuple the output blocks are y_f = sum_e Gamma[f][e] x_e (legs
 * permuted), Gamma composed on the host in FP64 (see sym_su2_chain_gamma),
 * the combination on the device in FP64 on FP32 data.  in: SU(2), FP32, on
 * the CHAIN, OPERATOR or LEFT tree, any layout; n_row_out: any layout the
 * CHAIN tree allows.  Limits: rank <= 8, at most 32 blocks per label tuple
 * (SYM_E_UNSUPPORTED otherwise).  sym_su2_permute_output creates the result's
 * handle (data may be NULL); sym_su2_permute writes into out, which must
 * describe exactly that result; in and out must not overlap.  The plan is
 * built on the first call and cached. */
int32_t sym_su2_permute_output(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, const int32_t* arrows_out,
                               int32_t n_row_out, void* data, sym_tensor** out);
int32_t sym_su2_permute(sym_ctx* ctx, const sym_tensor* in, const int32_t* perm, const int32_t* arrows_out,
                        int32_t n_row_out, sym_tensor* out, void* stream);
/* FUSE and SPLIT of two adjacent legs of an SU(2) tensor (section "Reshape
 * of indices" of the tree-decomposition chapter; eq:fuse, eq:su2fusecanon).
 * FUSE: legs leg and leg + 1 of in (one arrow) become one leg whose labels
 * are every spin c of j_a (x) j_b, with degeneracy the sum of d_a d_b over the
 * pairs (j_a, j_b) that reach c; inside c the pairs run lexicographically
 * (j_a, then j_b), each over its d_a x d_b degeneracy indices row-major.
 * When the two legs are the first two of their chain, the fusion deletes the
 * first node and moves no value (the blocks are relabelled); otherwise one
 * F-move (eq:fmove2, FP64) maps their two nodes to (A, c -> J).  SPLIT is the
 * inverse: leg `leg` of in, the fusion of legs2[0] and legs2[1] (their
 * labels and degeneracies; arrows are taken from in's leg, SYM_E_SPECTRUM if
 * they do not fuse to it), becomes those two legs.  in: SU(2), FP32, CHAIN
 * tree (FUSE also takes OPERATOR and LEFT), any layout; the result is on the
 * CHAIN tree with n_row_out.  *_output create the result's handle (data may
 * be NULL); sym_su2_fuse / sym_su2_split write into out, which must describe
 * exactly that result; in and out must not overlap.  Plans are cached. */
int32_t sym_su2_fuse_output(sym_ctx* ctx, const sym_tensor* in, int32_t leg, int32_t n_row_out, void* data,
                            sym_tensor** out);
int32_t sym_su2_fuse(sym_ctx* ctx, const sym_tensor* in, int32_t leg, int32_t n_row_out, sym_tensor* out,
                     void* stream);
int32_t sym_su2_split_output(sym_ctx* ctx, const sym_tensor* in, int32_t leg, const sym_leg* legs2, int32_t n_row_out,
                             void* data, sym_tensor** out);
int32_t sym_su2_split(sym_ctx* ctx, const sym_tensor* in, int32_t leg, sym_tensor* out, void* stream);
/* Spectrum of leg `leg` of a tensor: *n labels, their degeneracies and the
 * arrow.  With labels and degs both NULL only *n (and *arrow) are written;
 * otherwise SYM_E_ARG if *n is above cap. */
int32_t sym_tensor_leg(const sym_tensor* t, int32_t leg, int32_t cap, int32_t* n, int32_t* labels, int64_t* degs,
                       int32_t* arrow);

/* The Gamma of sym_permute_tree for one label tuple, on the host: spins[4]
 * are the doubled spins of the input's legs; on return *n is the number of
 * intermediate spins, es[*n] the input tree's (ascending), fs[*n] the output
 * tree's, gamma[f * n + e] the coefficients.  cap is the capacity of es and
 * fs (gamma holds cap * cap); SYM_E_ARG when *n would exceed it.  No GPU. */
int32_t sym_su2_gamma(int32_t tree_in, const int32_t* perm, int32_t tree_out, const int32_t* spins, int32_t cap,
                      int32_t* n, int32_t* es, int32_t* fs, double* gamma);

/* The Gamma of a PERMUTE with REVERSE between CHAIN trees for one label
 * tuple, on the host (eq:Gamma, eq:permsu2; section "Reversal of indices"):
 * input legs with arrows_in and doubled spins spins[rank]; output leg i is
 * input leg perm[i] with arrow arrows_out[i].  On return *n is the number of
 * blocks of the tuple (the same on both sides), keys_in[n * key_len_in] and
 * keys_out[n * key_len_out] their keys in block order (see
 * sym_tensor_block_inner), gamma[f * n + e] the coefficient from input block e
 * to output block f.  Composed in FP64 from exchanges at a node (eq:braid3),
 * F-moves (eq:fmove2, 6j by Racah's formula) and bends (eq:cupj, eq:capj; the
 * leg's m index summed against the cup's or cap's row index).  cap bounds n
 * (keys hold cap * rank entries, gamma cap * cap); SYM_E_ARG when n exceeds
 * it.  No GPU. */
int32_t sym_su2_chain_gamma(int32_t rank, const int32_t* arrows_in, const int32_t* perm, const int32_t* arrows_out,
                            const int32_t* spins, int32_t cap, int32_t* n, int32_t* key_len_in, int32_t* key_len_out,
                            int32_t* keys_in, int32_t* keys_out, double* gamma);

/* Handle of a contraction's operand in the layout the grouped GEMM reads
 * (which = 0: A's legs in the order free legs, then axesA, its free legs the
 * rows; which = 1: B's legs in the order axesB, then free legs, its sector
 * matrices stored transposed), in the compute type, rows padded to 128-byte
 * lines and sector bases to 64 elements: the fused operand of eq:multi2.
 * A tensor in this layout, contracted over its last (A) or first (B) legs in
 * order, is read in place by sym_contract and its relatives (no fuse, no
 * workspace), so an operand reused across many contractions is fused once.
 * Its padding entries must be zero (allocate the buffer zeroed); fill it with
 * sym_permute_fuse, which writes only its blocks; its data must be 256-byte
 * aligned.  A contraction's C may also be such a handle when the next
 * contraction takes it as operand A in compute F32: the GEMM then writes it
 * directly.  Abelian groups and the rank-4 SU(2) operator form; data may be
 * NULL. */
int32_t sym_contract_operand_output(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                                    const int32_t* axesA, const int32_t* axesB, int32_t compute, int32_t which,
                                    void* data, sym_tensor** out);

/* Contraction C = A . B (see above).  compute: SYM_F32 (FP32 MFMA, FP32
 * accumulate) or SYM_BF16 (operands rounded to BF16 on the device, BF16 MFMA,
 * FP32 accumulate, FP32 output).  C must have dtype F32.  Small Abelian
 * contractions (FP32 throughout, no fermionic signs, at most 2^25 useful
 * FLOPs over the call, every block of A, B and C a strided matrix over its
 * row and column legs) run as one kernel launch that reads the operand
 * blocks in place and sums each output block over its block pairs
 * (eq:tensormult) in FP32 fused multiply-adds; the environment variable
 * SYM_SMALL=off (read when a plan is built) sends them through the fuse /
 * grouped GEMM / split path instead.  SU(2): an OPERATOR
 * tensor A contracted on legs (2,3) with legs (0,1) of an OPERATOR or LEFT
 * tensor B gives C on B's tree (sector-major, n_row 2), by one GEMM per
 * intermediate spin (any compute type).  Any other SU(2) contraction of
 * CHAIN, OPERATOR or LEFT tensors, over any axes (at least one contracted and
 * one free leg on each side), follows the five steps of the thesis on CHAIN
 * trees (section "Multiplication of two tensors" of the tree-decomposition
 * chapter): A is recoupled (PERMUTE with REVERSE, sym_su2_permute) so that its
 * free legs are incoming rows and its contracted legs outgoing, B so that its
 * contracted legs (in the order of axesB) are incoming rows, one GEMM runs per
 * coupled spin of the contracted legs (the Clebsch-Gordan chains of the
 * contracted legs contract to the identity, eq:cgunitary), and the product is
 * recoupled into C, a CHAIN tensor (default layout: the canonical block list)
 * with A's free legs then B's free legs and their arrows.  Compute F32 needs
 * FP32 operands; with SYM_BF16 the recoupling of A and B (FP32 or BF16 data,
 * FP64 sums) writes their GEMM forms rounded once to BF16, and the product
 * is recoupled from FP32 into C.  sym_contract_output creates C's handle
 * (data may be NULL).  The plan (block matching, offsets, tile list) is built
 * on the first call and cached in the context. */
int32_t sym_contract_output(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                            const int32_t* axesA, const int32_t* axesB, void* data, sym_tensor** C);
int32_t sym_contract(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                     const int32_t* axesA, const int32_t* axesB, int32_t compute, sym_tensor* C,
                     void* stream);

/* sym_contract for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bit for bit) as sym_contract; the
 * difference is where the library's own device memory lives.  Instead of
 * workspaces from the context's allocator, the fused operands, any split
 * workspace and the plan's tables are placed in a fixed array of
 * sym_noalloc_capacity() bytes (64 MiB) that the library holds on every
 * device it runs on until the process ends.  No call allocates or frees
 * device memory (the host plan is built on the first call per structure and
 * cached in the context, host memory only).
 * Limit: a contraction whose fused operands, split workspace and tables need
 * more than the array holds fails with SYM_E_UNSUPPORTED before any launch.
 * All calls on one device share the array and find it as the last call left
 * it: each call first re-uploads its tables (asynchronous copies on
 * `stream`) and clears the fused-operand workspace with a kernel.  Calls that
 * overlap in time on one device (any context, any stream) race on the array
 * and must not be made. */
int32_t sym_contract_noalloc(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                             const int32_t* axesA, const int32_t* axesB, int32_t compute, sym_tensor* C,
                             void* stream);
int32_t sym_noalloc_capacity(int64_t* bytes);

/* Backward of C = A . B for a cotangent dC (same description as C): per
 * sector dA_s = dC_s B_s^T and dB_s = A_s^T dC_s, split back into A's and B's
 * layouts (the adjoint of eq:blockmult).  dA or dB may be NULL to skip it;
 * given ones must describe A and B (dtype F32). */
int32_t sym_contract_backward(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B,
                              const sym_tensor* dC, int32_t n, const int32_t* axesA,
                              const int32_t* axesB, int32_t compute, sym_tensor* dA, sym_tensor* dB,
                              void* stream);

/* count (any number >= 1) independent contractions C[i] = A[i] . B[i] with
 * the same axes: all fuses in one launch, every sector GEMM of every member in
 * one persistent grouped-GEMM launch, all splits in one launch, per chunk of
 * 64 members (device pointers travel as kernel arguments, 3 per member); every
 * chunk is validated before the first launch, so a bad member anywhere
 * leaves every output untouched. */
int32_t sym_contract_batched(sym_ctx* ctx, int32_t count, const sym_tensor* const* A,
                             const sym_tensor* const* B, int32_t n, const int32_t* axesA,
                             const int32_t* axesB, int32_t compute, sym_tensor* const* C,
                             void* stream);

/* Useful work of a contraction: sum over sectors of 2 M_s N_s K_s. */
int32_t sym_contract_flops(sym_ctx* ctx, const sym_tensor* A, const sym_tensor* B, int32_t n,
                           const int32_t* axesA, const int32_t* axesB, int64_t* flops);

/* HIP graph of a batched contraction of any count: captured once on `stream`
 * (the plans, one per chunk of 64 members, are built first, outside the
 * capture), replayed with sym_graph_launch.  A contraction small enough to
 * run as one kernel (see sym_contract) is not captured: its replay launches
 * that kernel with the arguments fixed here, which costs less than a graph
 * launch.  The tensors' data pointers must stay valid and unchanged while
 * the graph lives. */
int32_t sym_graph_create_batched(sym_ctx* ctx, int32_t count, const sym_tensor* const* A,
                                 const sym_tensor* const* B, int32_t n, const int32_t* axesA,
                                 const int32_t* axesB, int32_t compute, sym_tensor* const* C,
                                 void* stream, sym_graph** out);
int32_t sym_graph_launch(sym_graph* g, void* stream);
void sym_graph_destroy(sym_graph* g);

/* Kernel timing of the most recent batched contraction on a context, when
 * enabled with sym_ctx_set_timing(ctx, 1): HIP events recorded on the launch
 * stream around each phase; times in milliseconds, valid after the stream is
 * synchronised.  phase: 0 = fuse, 1 = grouped GEMM, 2 = split. */
int32_t sym_ctx_set_timing(sym_ctx* ctx, int32_t enable);
int32_t sym_ctx_phase_ms(sym_ctx* ctx, int32_t phase, float* ms);

/* Tile configuration the grouped GEMM uses for a compute type, and the
 * autotuner's entry point (at most 64 contractions): the plan of this
 * contraction is built once and run once (its fused operands written); each
 * compiled tile variant then gets its own tile list over the same plan and
 * one timed GEMM launch, the (at most five) fastest within 8 % of the
 * fastest and the default three more, each right after the plan's fuse as
 * in a call, taken round-robin, and the smallest sum wins unless the
 * default variant is within 1 % of it.  When the default variant's tile
 * list has at least eight tiles per CU, variants whose tiles cover a
 * quarter of the default's area or less are not timed.  The winner becomes
 * the cached plan of the structure (also written to the file named by
 * SYM_TUNE_CACHE, when set).  Writes C. */
int32_t sym_tune_batched(sym_ctx* ctx, int32_t count, const sym_tensor* const* A,
                         const sym_tensor* const* B, int32_t n, const int32_t* axesA,
                         const int32_t* axesB, int32_t compute, sym_tensor* const* C, void* stream,
                         int32_t* best_variant);
int32_t sym_ctx_set_variant(sym_ctx* ctx, int32_t compute, int32_t variant);
int32_t sym_num_variants(int32_t compute, int32_t* count);
/* Name of a tile variant (static storage, never freed), and the variant a
 * context uses for a compute type when nothing was set or tuned. */
int32_t sym_variant_name(int32_t compute, int32_t variant, const char** name);
/* The kernel a tile variant launches, as its template instance (for example
 * "k_gemm_bf16_dl<256, 256, 32, 2, 4, 5, 2>"), the form profilers print
 * inside the kernel's full name.  Static string; host only. */
int32_t sym_variant_kernel(int32_t compute, int32_t variant, const char** kernel);
int32_t sym_default_variant(int32_t compute, int32_t* variant);

/* Block-wise singular value decomposition (section "Factorization of a
 * matrix" of the symmetric tensor network chapter; eq:svd0, eq:svd1): every
 * sector matrix T_s of T's layout (rows = T's first n_row legs, M_s x N_s) is
 * factorised independently in FP64 as T_s = U_s diag(s_s) Vt_s, k_s =
 * min(M_s, N_s), singular values descending.  U, S, Vt are FP64 device
 * buffers, sector after sector in T's sector order (sectors with no rows or
 * no columns skipped): U_s row-major M_s x k_s, s_s k_s values, Vt_s row-major
 * k_s x N_s; sym_svd_sizes gives their element counts.  One-sided Jacobi with
 * plane rotations, all sectors together, until a sweep rotates nothing
 * (for every pair of vectors of length L, |a.b| <= sqrt(L) 2^-53 |a||b|
 * or |a.b| below 1e-30 of the sector's squared Frobenius norm) or max_sweeps sweeps; sweeps (host,
 * may be NULL) receives the number run.  The call synchronises `stream` once
 * per sweep (the stopping decision is taken on the host).  Singular vectors
 * of zero singular values are returned as zeros.  SYM_E_UNSUPPORTED for a
 * sector with min(M_s, N_s) > 4096.  A tensor with no sector (all three
 * sizes 0) returns at once: U, S, Vt may then be NULL, and *sweeps is 0.
 * The caller owns the outputs; the FP64
 * workspaces belong to the context (cached per structure), so calls on one
 * structure must not overlap. */
int32_t sym_svd_sizes(const sym_tensor* T, int64_t* u_elems, int64_t* s_elems, int64_t* vt_elems);
int32_t sym_svd(sym_ctx* ctx, const sym_tensor* T, double* U, double* S, double* Vt, int32_t* sweeps,
                int32_t max_sweeps, void* stream);
/* Block-wise symmetric eigen-decomposition (section "Factorization of a
 * matrix" of the symmetric tensor network chapter, where an eigen-
 * decomposition factorises a tensor block by block the same way as eq:svd1):
 * every sector matrix of T's layout must be square (k_s x k_s;
 * SYM_E_UNSUPPORTED otherwise, and for k_s > 4096), and the routine
 * factorises its symmetric part S_s = (T_s + T_s^T) / 2 in FP64 as
 * S_s = V_s diag(w_s) V_s^T, eigenvalues descending, V_s orthonormal.  V and
 * w are FP64 device buffers, sector after sector in T's sector order
 * (sectors with no rows skipped): V_s row-major k_s x k_s with the
 * eigenvectors as columns, w_s k_s values; sym_eigh_sizes gives their
 * element counts.  Method: S_s + c_s I, c_s the Frobenius norm of S_s (1 when
 * S_s = 0), is positive definite, so the one-sided Jacobi SVD of sym_svd
 * (same stopping rule, same once-per-sweep synchronisation of `stream`)
 * returns its eigenvectors, taken from the accumulated rotations, and
 * eigenvalues w = s - c_s; the absolute error of an eigenvalue is a small
 * multiple of sqrt(k_s) 2^-53 c_s.  sweeps (host, may be NULL) receives the
 * number of sweeps.  A tensor with no sector returns at once (V, w may be
 * NULL).  The caller owns the outputs; the workspaces belong to the context,
 * so calls on one structure must not overlap. */
int32_t sym_eigh_sizes(const sym_tensor* T, int64_t* v_elems, int64_t* w_elems);
int32_t sym_eigh(sym_ctx* ctx, const sym_tensor* T, double* V, double* w, int32_t* sweeps, int32_t max_sweeps,
                 void* stream);
/* Block-wise polar decomposition (section "Factorization of a matrix": like
 * the spectral decomposition, it is obtained by factorising every block on
 * its own): each sector matrix T_s (M_s x N_s, rows = T's first n_row legs)
 * is written as T_s = W_s P_s when M_s >= N_s, or T_s = P_s W_s when
 * M_s < N_s, with W_s = U_s Vt_s (M_s x N_s, orthonormal columns or rows)
 * and P_s = V_s diag(s_s) Vt_s or U_s diag(s_s) U_s^T (k_s x k_s, symmetric
 * positive semidefinite), from the block SVD of sym_svd (same method and
 * stopping rule, same once-per-sweep synchronisation of `stream`) followed
 * by FP64 products on the device.  W and P are FP64 device buffers, sector
 * after sector in T's sector order (sectors with no rows or no columns
 * skipped), row-major; sym_polar_sizes gives their element counts.  P may be
 * NULL (only W is written).  For a rank-deficient sector W_s is zero on the
 * null space (the singular vectors of zero singular values are zero), so it
 * is a partial isometry.  sweeps (host, may be NULL) receives the number of
 * sweeps.  SYM_E_UNSUPPORTED for a sector with min(M_s, N_s) > 4096.  The
 * U, S and Vt workspaces belong to the context, so calls on one structure
 * must not overlap. */
int32_t sym_polar_sizes(const sym_tensor* T, int64_t* w_elems, int64_t* p_elems);
int32_t sym_polar(sym_ctx* ctx, const sym_tensor* T, double* W, double* P, int32_t* sweeps, int32_t max_sweeps,
                  void* stream);
/* Global truncation of a block SVD (host; S is a host copy of sym_svd's S):
 * the singular values of all sectors are taken in descending order, each
 * counting w_s times (1 for the Abelian groups, 2e + 1 for the SU(2) sector
 * of coupled spin e: the multiplicity of s_s in the SVD of the full matrix),
 * and kept while the running total stays within chi_max and the value
 * exceeds tol; the first value that does not fit ends the cut.  keep[i]
 * (one per sector of T, 0 for skipped sectors) receives the number kept in
 * sector i; discarded (may be NULL) the sum of w_s s^2 over dropped values,
 * the squared Frobenius norm of the truncation error. */
int32_t sym_svd_truncate(const sym_tensor* T, const double* S, int64_t chi_max, double tol, int32_t* keep,
                         double* discarded);

/* SU(2) recoupling coefficient F^{jD jE}_{jA jB jC jJ} (eq:sixj), doubled
 * spins, from the library's own tables: Racah's sum taken exactly, then
 * rounded to FP64.  Spins up to 60 (doubled 120); above that the result is
 * NaN and sym_last_error says why.  Host only. */
double sym_fmove_coeff(int32_t tjA, int32_t tjB, int32_t tjC, int32_t tjJ, int32_t tjD, int32_t tjE);

const char* sym_last_error(void);
const char* sym_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SYMTENSOR_H */
