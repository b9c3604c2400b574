// Structures shared by the host planner and the HIP kernels.
//
// A block state of q qubits evolved for P = 2^p paths at once is stored as
// one array of 2^(p+q) complex numbers, "extended index" e = i*P + slot:
// the slot (path) bits are the p lowest bits and qubit t is bit p+t.  The
// slot axis behaves like p extra low qubits that no gate touches, so every
// gate sees contiguous runs of P amplitudes (coalesced HBM access) and the
// gather reads one contiguous row of P values per requested index.
//
// A "pass" streams the whole array once.  A wave owns a tile of 64 * 2^R
// amplitudes: lane l holds the 2^R amplitudes whose 6 lowest extended bits
// equal l and whose R "register bits" (chosen qubits) run over all values;
// the remaining bits come from the tile index.  Gates on register qubits are
// applied in registers, gates on the (up to 6) qubits that sit in lane bits
// with cross-lane shuffles, and diagonal gates (CZ, T, and the per-path
// projector / Z of crossing gates, Section 2 Eq. (CZ)) as bitmask phase
// evaluations (the paper's bitmask + mod-8 arithmetic of Section 2).  The
// per-path flips of crossing iSWAPs are register swaps or lane shuffles.
#pragma once
#include <stdint.h>

namespace sf {

// One-qubit gate kinds applied by the kernels (unnormalised forms):
//   H' = [[1,1],[1,-1]]          H     = H' / sqrt2
//   X' = [[1,-i],[-i,1]]         X^1/2 = X' (1+i)/2
//   Y' = [[1,-1],[1,1]]          Y^1/2 = Y' (1+i)/2
// Each primed form has norm gain sqrt2; the host tracks the scalars and
// folds exact powers of two back in ("rescaling").
enum GateKind : uint8_t { GK_H = 0, GK_X = 1, GK_Y = 2 };

// PO_PFLIP_*: the non-diagonal branch operator of a crossing iSWAP (Eq. (4way)): flip the target
// qubit in the slots whose path bits u and u+1 differ, and (kind 1) multiply those slots by i.
// PO_ISWAP: an iSWAP between two qubits of the block held in the pass's registers or lanes;
// target and group (low byte) give the two positions (register index or lane bit) and kind bit 0
// (bit 1) says that the target (group) position is a lane bit.
enum PassOpType : uint8_t { PO_REG = 0, PO_LANE = 1, PO_DIAG = 2, PO_PFLIP_REG = 3, PO_PFLIP_LANE = 4, PO_ISWAP = 5 };

struct PassOp {
    uint8_t type;    // PassOpType
    uint8_t kind;    // GateKind for PO_REG / PO_LANE; 1 = with the factor i for PO_PFLIP_*
    uint8_t target;  // register index k (PO_REG, PO_PFLIP_REG) or lane bit b (PO_LANE, PO_PFLIP_LANE)
    uint8_t pad;
    uint32_t group;  // diagonal group index (PO_DIAG); path bit u (PO_PFLIP_*)
};

// A merged set of commuting diagonal operators, evaluated per amplitude as
//   keep(e) * omega^{m(e)},  omega = e^{i pi/4},
//   m(e) = sum_lin w * e_b + 4 sum_quad e_a e_b + 4 sum_zs e_b s_u   (mod 8)
//   keep(e) = prod_proj [e_a == s_u]
// where e_x is bit x of the extended index and s_u bit u of the slot's path
// id.  Terms are pre-split by whether their bits are register bits ("r",
// given by register index k) or base bits ("b", extended bit position).
struct DiagGroup {
    uint16_t n_lin_b, n_quad_bb, n_quad_br, n_zs_b, n_zs_r, n_proj_b, n_proj_r;
    uint16_t flags;            // bit 0: some weight not a multiple of 4; bit 1: has projectors;
                               // bit 2 (3): some register entry of tab has bit 0 (bit 1) set
    uint32_t term_off;         // offset (in byte pairs) into the term array
    uint32_t pad;
    uint64_t tab[4];           // m contribution of register-only terms, 4 bits per j < 64
};
// term layout (pairs of bytes), in this order:
//   lin_b  (bit, weight)   quad_bb (bit_a, bit_b)   quad_br (bit_a, k)
//   zs_b   (bit_b, u)      zs_r    (k, u)           proj_b  (bit_a, u)   proj_r (k, u)

enum SrcMode : int32_t { SRC_SAME = 0, SRC_INIT = 1, SRC_FANOUT = 2 };

// A pass program (ops, then diagonal groups, then term bytes) is one
// contiguous block of at most kMaxProgWords 32-bit words; the kernel stages
// it in LDS once per workgroup so the per-tile interpreter never touches
// global memory for it.
constexpr int kMaxProgWords = 2048;
// Most known-zero entries a pass carries (a subset of the true zeros is always valid).
constexpr int kMaxZeroEntries = 4;

struct PassArgs {
    void *dst;
    const void *src;
    const uint64_t *slot_path;    // per destination slot: path id of the node (low bits 0 below its level)
    const uint32_t *slot_parent;  // per destination slot: slot of its parent in src (SRC_FANOUT)
    const uint32_t *prog;         // pass program in global memory
    // Rows the path sum reads (nullptr: all).  Bit b of row_mask says whether the tiles whose
    // block-qubit bits (extended index >> p_dst, zero at the qubits inside a tile) equal b hold
    // an amplitude the gather or fold reads; the others are neither read nor written.  Only the
    // last pass of a block at the level the gather reads carries it.
    const uint32_t *row_mask;
    uint32_t prog_words;          // its size
    uint32_t groups_word;         // word offset of the DiagGroup array (8-byte aligned)
    uint32_t terms_word;          // word offset of the term bytes
    uint64_t n_tiles;             // 2^(n_ext - 6 - R)
    uint64_t init_zero_mask;      // SRC_INIT: extended bits that must be 0 for a non-zero amplitude
    double rescale;               // multiply every amplitude by this at the end (exact power of 2)
    uint32_t n_ops;
    uint32_t slot_parent_base;    // SRC_FANOUT: parent slot = slot_parent[slot] - slot_parent_base
    int32_t p_dst, p_src;         // slot bits of destination and source
    int32_t src_mode;
    int32_t reg_pos[6];           // extended bit positions of register bits, ascending
    // Tile enumeration: the n_low lowest bits of a tile index go to extended bits low_pos[]
    // (sibling bits of a fan-out, so the children of one parent are handled by neighbouring
    // waves and the parent is read from cache), the other tile bits fill the remaining free
    // bits in ascending order.  skip_pos = register and low positions, ascending.
    int32_t n_low, n_skip;
    int32_t low_pos[4];
    int32_t skip_pos[10];
    // Known zeros of the source state (zero-subspace skipping): the amplitude at extended
    // index e is zero unless, for every entry k < n_zero, the bit of e that holds qubit
    // zero_pos[k] (destination layout) equals bit zero_bit[k] of the slot's path id.  Entries
    // with zero_reg[k] >= 0 sit on register bit zero_reg[k]; the others on lane or tile bits.
    // A kernel built for it leaves such amplitudes unread; any other kernel ignores the list.
    // Slots in use (the rest pad the batch to a power of two; 0 = all): a tile whose 64 slots
    // all lie beyond them is neither read nor written.  Lanes and registers never mix slots, so
    // padding never reaches a slot in use.
    uint64_t slots_real;
    // Lane bits: with lane_qpos = 0 the 6 lowest extended bits; otherwise (every lane bit would be
    // a slot bit, p_dst >= 6) lane bit 5 holds extended bit lane_qpos (a qubit), and with
    // lane_qpos4 > 0 lane bit 4 holds extended bit lane_qpos4 too, so a pass applies gates to one
    // or two more qubits; each load and store then covers two runs of 32 (four of 16) consecutive
    // amplitudes.  The displaced slot bits come from the tile index; the positions are in skip_pos.
    int32_t lane_qpos;
    int32_t lane_qpos4;
    int32_t n_zero;
    int8_t zero_reg[kMaxZeroEntries];
    uint8_t zero_pos[kMaxZeroEntries];
    uint8_t zero_bit[kMaxZeroEntries];
};

// A run of small dependent passes in one persistent launch (pass_chain_kernel): phase i runs
// args[first] on every workgroup, or (n = 2, the two blocks' independent passes) args[first] on
// workgroups [0, split) and args[first + 1] on the rest; a grid barrier separates the phases.
struct ChainPhase {
    uint32_t first;
    uint32_t n;
    uint32_t split;
    uint32_t pad;
};

// Dense fused block: a 2^4 x 2^4 complex matrix U applied to four qubits (extended bit
// positions bpos[0] < ... < bpos[3], all >= 5), on matrix cores.  `mat` is the real
// embedding [[Ur, -Ui], [Ui, Ur]] (32 x 32, row-major, FP32).  The 5 lowest extended
// bits index 32 columns that are contiguous in memory.
struct DenseArgs {
    void *dst;
    const void *src;
    const float *mat;
    uint64_t n_groups;            // 2^(n_ext - 9): groups of 32 columns
    double rescale;
    int32_t bpos[4];
    int32_t p;                    // slot bits
    uint64_t slots_real;          // slots in use (0 = all): groups of padding slots are skipped
};

struct GatherArgs {
    const void *a;                // block-A leaf states, 2^(p+qA) complex
    const void *b;                // block-B leaf states, 2^(p+qB) complex
    const uint32_t *xa, *xb;      // per bitstring: x_A, x_B
    const uint32_t *order;        // visiting order of the bitstrings (NULL = as given)
    double *acc;                  // 2 * n_bits doubles (re, im), accumulated
    uint64_t n_bits;
    uint32_t n_slots;             // real slots (<= 2^p)
    int32_t p;
    double scale_re, scale_im;    // product of both blocks' tracked scalars
};

// Fold of the last F tree levels: the gather reads level L-F and applies the F levels itself.
// The nb path bits these levels decide index the "virtual slots" i of a descendant; path bit u
// belongs to a branch operator on local qubit bq[u].  For block h and output bits x (local):
//   c_h[i] = [ bits u of i outside S equal x at bq[u] ] * tab[pext(x, tmask) * 2^n_s + y(i)]
//            * parent_h[(x & ~smask) + sum_u i_u * sstride[u]][slot],
//   y(i) = sum over u with bq[u] in S of i_u << ypos[u]   (i's S pattern, an index of tab's row).
// Block A's projectors keep exactly descendant i; block B's Z^b signs become a Walsh-Hadamard
// transform over i.  Then amp[x] += scale * sum_slot sum_{i in child_mask[slot]} c_A[i] c_B'[i]
// with c_B' = WHT(c_B).
struct FoldHalf {
    const void *par;              // states of the block at level L-F, 2^(p+q) complex
    const double *tab;            // complex (re, im) table of V, [2^|T|][2^n_s]
    uint32_t smask, tmask;        // local qubits of S (non-diagonal gates), of T (all of V)
    uint32_t dsel;                // bit u set if bq[u] is outside S
    int32_t n_s;
    uint32_t sstride[5];          // 1 << bq[u] if bq[u] is in S, else 0
    uint8_t bq[5];
    uint8_t ypos[5];              // S index of bq[u] (unused if outside S)
    uint8_t pad[6];
};

struct FoldArgs {
    FoldHalf h[2];
    const uint32_t *xa, *xb;      // per bitstring: x_A, x_B
    const uint32_t *order;        // visiting order of the bitstrings
    const uint32_t *child_mask;   // per parent slot: bit i set if descendant i is requested
    double *acc;                  // 2 * n_bits doubles, accumulated
    uint64_t n_bits;
    uint32_t n_slots;             // real parent slots (<= 2^p)
    int32_t p;                    // parent slot bits
    int32_t all_children;         // 1: every parent slot has all 2^nb descendants (masks not read)
    double scale_re, scale_im;
};

// General fold of the last F tree levels (CZ branch operators only), for levels whose
// non-diagonal gates also act on qubits other than their branch qubits.  S' = the qubits of the
// non-diagonal gates plus the nb branch qubits, T' = S' plus the qubits the levels' diagonal
// gates touch.  A column index y' of S' patterns holds the branch values in its nb low bits (bit
// u = the qubit of path bit u) and the other S' qubits above them in ascending order.  For block
// h, output bits x (local) and descendant branch value b:
//   w_h[b] = sum_{r < 2^(|S'|-nb)} tab[pext(x, tmask) * 2^|S'| + (b | r << nb)]
//                                  * parent_h[(x & ~smask) | off[b | r << nb]][slot]
// Block A's projectors keep exactly the column patterns whose branch bits equal b, so
// c_A[b] = w_A[b]; block B's Z^b signs give c_B = WHT(w_B) over b.  Then
// amp[x] += scale * sum_slot sum_{b in child_mask[slot]} c_A[b] c_B[b].
struct GFoldHalf {
    const void *par;              // states of the block at level L-F, 2^(p+q) complex
    const void *tab;              // table of V in the state precision (complex), [2^|T'|][2^|S'|]
    const uint32_t *off;          // per column pattern y': its S' bits placed at their local qubits
    uint32_t smask, tmask;        // local qubits of S', of T'
    int32_t n_s;                  // |S'|
    int32_t n_rest;               // |S'| - nb
    // Deferred level (block A, par_slot != nullptr): par is the batch of the level above (2^p_par
    // slots); gather slot s reads parent slot par_slot[s] at the rows with the projected qubits
    // (dmask) set to dsub[s], and its sums are multiplied by dfac[s * 2^nd + pext(x, dmask)]
    // (complex, state precision): the entry of the deferred one-qubit gates.
    const uint32_t *par_slot;
    const uint32_t *dsub;
    const void *dfac;
    uint32_t dmask;
    int32_t p_par;
    int32_t nd;
    int32_t pad;
};

struct GFoldArgs {
    GFoldHalf h[2];
    const uint32_t *xa, *xb;      // per bitstring: x_A, x_B
    const uint32_t *order;        // visiting order of the bitstrings
    const uint32_t *child_mask;   // per parent slot: bit b set if descendant b is requested
    double *acc;                  // 2 * n_bits doubles, accumulated
    uint64_t n_bits;
    uint32_t n_slots;             // real parent slots (<= 2^p)
    int32_t p;                    // parent slot bits
    int32_t all_children;         // 1: every parent slot has all 2^nb descendants (masks not read)
    int32_t pad;
    double scale_re, scale_im;
};

// Fold of trailing levels whose crossing gates are all iSWAPs (G of them, Eq. (4way)).  Gate g
// decides path bits u[g] (j) and u[g]+1 (i) of the descendant; block A takes |i><j| = X^{i^j} P_j
// and block B G_ij = i^{i^j} X^{i^j} P_i on qubit q[g].  For a block, a pattern t of G bits (bit g
// = the branch value feeding V's column: i on A, j on B; the parent row takes the other value,
// written r below) gives
//   V_h(t) = [ x at q[g] equals t_g for every g outside S ] * tab[pext(x, tmask) * 2^n_s + y(t)],
//   row_h(r) = parent_h[(x & ~qmask) | sum_g r_g << q[g]][slot],
// and the descendant (i, j) adds V_A(i) row_A(j) * V_B(j) row_B(i) * i^{popcount(i ^ j)}.
struct FoldIswapHalf {
    const void *par;              // states of the block at level L-F, 2^(p+q) complex
    const double *tab;            // complex (re, im) table of V, [2^|T|][2^n_s]
    uint32_t qmask, tmask;        // local qubits of the gates, of T (all of V)
    int32_t n_s;
    uint8_t q[4];                 // local qubit of gate g
    int8_t ypos[4];               // S index of q[g], -1 if q[g] is outside S
    uint32_t pad;
};

struct FoldIswapArgs {
    FoldIswapHalf h[2];
    const uint32_t *xa, *xb;      // per bitstring: x_A, x_B
    const uint32_t *order;        // visiting order of the bitstrings
    const uint64_t *child_mask;   // per parent slot: bit v set if descendant v is requested
    double *acc;                  // 2 * n_bits doubles, accumulated
    uint64_t n_bits;
    uint32_t n_slots;             // real parent slots (<= 2^p)
    int32_t p;                    // parent slot bits
    int32_t all_children;         // 1: every parent slot has all descendants (masks not read)
    uint8_t u[4];                 // lower path bit of gate g among the folded bits
    double scale_re, scale_im;
};

}  // namespace sf
