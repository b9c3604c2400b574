// Host-side data structures: circuit, cut, per-block programs and pass plans.
#pragma once
#include <complex>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/sfpath.h"
#include "sf_device.hpp"

namespace sf {

// Operations of one block's program, in local qubit indices.
enum HalfKind : uint8_t {
    HK_H = 0, HK_X = 1, HK_Y = 2, HK_T = 3, HK_CZ = 4,
    HK_PROJ = 5,   // keep amplitudes whose bit q0 equals path bit `bit` (crossing CZ block A side; both sides of an iSWAP)
    HK_ZCTL = 6,   // negate amplitudes whose bit q0 is 1 when path bit `bit` is 1 (block B side)
    HK_PFLIP = 7,  // flip bit q0 when path bits bit and bit+1 differ (crossing iSWAP, X^{i xor j})
    HK_PFLIPI = 8, // as HK_PFLIP, and multiply by i when it flips
    HK_ISWAP = 9,  // iSWAP on q0, q1 inside the block: |01> -> i|10>, |10> -> i|01> (Section 7)
};

struct HalfOp {
    uint8_t kind;
    uint8_t q0, q1;
    uint8_t bit;   // path bit index u (bit u of the path id): HK_PROJ / HK_ZCTL, lower bit of HK_PFLIP(I)
};

inline bool is_diag(uint8_t k) { return k == HK_T || k == HK_CZ || k == HK_PROJ || k == HK_ZCTL; }
// operations on two local qubits (q0 and q1)
inline bool is_two_qubit(uint8_t k) { return k == HK_CZ || k == HK_ISWAP; }
// operators that depend on the path id (branch operators of crossing gates)
inline bool is_branch(uint8_t k) { return k == HK_PROJ || k == HK_ZCTL || k == HK_PFLIP || k == HK_PFLIPI; }
// the unnormalised one-qubit forms, whose norm gain sqrt2 the host tracks and rescales
inline bool has_gain(uint8_t k) { return k == HK_H || k == HK_X || k == HK_Y; }

// One pass of a segment: kernel ops plus the register-bit choice.
struct PassPlan {
    int R = 0;                      // register bits used
    int reg_pos[6] = {0, 0, 0, 0, 0, 0};
    std::vector<PassOp> ops;
    std::vector<DiagGroup> groups;
    std::vector<uint8_t> terms;
    int n_nondiag = 0;
    int rescale_exp = 0;            // divide by 2^rescale_exp at the end of the pass
    bool needs_slot_path = false;   // has path-dependent terms
    bool has_flip = false;          // has per-path flips (PO_PFLIP_*)
    // Zero subspace of the pass's input: (local qubit t, path bit u) pairs such that every
    // amplitude whose bit t differs from path bit u is zero (a projector on t applied, and no
    // non-diagonal gate on t since)
    std::vector<std::pair<uint8_t, uint8_t>> zero_in;
    std::vector<HalfOp> src;        // the block operations this pass applies, in program order
    int lane_q = -1;                // local qubit held by lane bit 5 (when the slots fill all lane bits)
    int lane_q4 = -1;               // local qubit held by lane bit 4 (only with lane_q)
    // dense pass (matrix cores): a 16 x 16 block on four qubits instead of the op list
    bool dense = false;
    int bpos[4] = {0, 0, 0, 0};     // extended bit positions, ascending
    std::vector<float> mat;         // 32 x 32 real embedding, row-major
};

// All passes of one block over one segment, for a given slot count 2^p.
struct SegmentPlan {
    std::vector<PassPlan> passes;
    bool ok = true;      // false if some operation could not be scheduled
};

// Most path bits the folded levels may decide (virtual slots per parent slot = 2^bits).
constexpr int kMaxFoldBits = 5;
// Most crossing iSWAPs the folded levels may hold (two path bits each).
constexpr int kMaxFoldGates = 3;
// General fold: most path bits (the kernel keeps 2 x 2^nb accumulators per lane), most S'
// qubits and most table bits |S'| + |T'| (the table goes to the plan blob in the state precision).
constexpr int kMaxGeneralFoldBits = 4;
constexpr int kMaxGeneralFoldS = 10;
constexpr int kMaxGeneralFoldTableBits = 16;

// The last F tree levels of one block written as V * D(b): D(b) = their branch operators for
// descendant branch value b (diagonal), V = the block's remaining gates of those levels
// (independent of b).  When every non-diagonal gate among them acts on a branch qubit, a
// descendant's amplitude at x is one amplitude of the level above per "virtual slot" i
// (descendant branch value i, see FoldHalf) times an entry of V, so the gather can read the
// level above and the states of the F levels are never written.
struct LeafFold {
    bool ok = false;
    int levels = 0;             // F
    int nb = 0;                 // path bits decided by the F levels
    int n_s = 0, n_t = 0;       // |S| (qubits of non-diagonal gates), |T| (all qubits V touches)
    uint32_t smask = 0, tmask = 0, dmask = 0;   // local masks of S, T, and branch qubits outside S
    int bq[kMaxFoldBits] = {0};                 // local qubit of the branch operator of path bit u
    int ypos[kMaxFoldBits] = {0};               // its index in S (-1 if outside S)
    std::vector<std::complex<double>> tab;      // [2^n_t][2^n_s]: <x_T| V |x_T with S bits := y>
    // iSWAP form (every branch operator a crossing iSWAP's projector + per-path flip): gate g
    // decides path bits gu[g] (j) and gu[g]+1 (i); its branch operators act on local qubit gq[g],
    // which feeds V's column with the branch value after the flip (index gy[g] in S, -1 if outside
    // S) and is read from the parent row with the value before it.  bq / ypos / dmask are unused.
    bool iswap = false;
    int ng = 0;
    int gq[kMaxFoldGates] = {0}, gu[kMaxFoldGates] = {0}, gy[kMaxFoldGates] = {0};
    uint32_t qmask = 0;                         // the gates' qubits (bits the parent row takes from the branch)
    // General form (GFoldArgs, CZ branch operators): S' = S plus the branch qubits, T' = T plus
    // the branch qubits, for levels whose non-diagonal gates also act on other qubits.  Available
    // when nb <= kMaxGFoldBits, the branch qubits are distinct and the table is small enough.
    // Columns y' hold the branch values in their nb low bits (bit u = path bit u) and the other
    // S' qubits above them in ascending order.
    bool gen_ok = false;
    int g_ns = 0, g_nt = 0;                     // |S'|, |T'|
    uint32_t g_smask = 0, g_tmask = 0;
    std::vector<std::complex<double>> gtab;     // [2^|T'|][2^|S'|]: <x_T'| V |x_T' with S' bits := y'>
    std::vector<uint32_t> goff;                 // per y': its S' bits at their local qubits
};

struct HalfProgram {
    int q = 0;                                  // qubits in the block
    uint64_t init_h_mask = 0;                   // local qubits whose opening H is folded into the initial state
    std::vector<std::vector<HalfOp>> segments;  // one per tree level (segment 0 = root)
    std::vector<std::complex<double>> seg_scale;  // scalar of each segment's unnormalised gates incl. rescaling
    std::vector<int> seg_rescale_exp;           // power of two divided out at the end of each segment
    std::complex<double> init_scale = 1.0;      // 2^{-h/2} for the folded opening H gates
    std::vector<LeafFold> folds;                // folds[F-1]: the last F levels as V * D(b)
};

struct Level {
    int cycle;          // clock cycle of this level's crossing gates
    int first_cut;      // index (in cut_gate) of its first crossing gate
    int n_cut;          // path bits its crossing gates decide (1 per CZ, 2 per iSWAP)
    int bits_after;     // path bits decided once this level's branch operators are applied
};

struct Circuit {
    int rows = 0, cols = 0, n = 0;
    std::vector<sf_gate_t> gates;

    // cut
    bool has_cut = false;
    uint64_t mask_a = 0, mask_b = 0;
    int k = 0;
    std::vector<int> cut_gate;        // gate index of crossing gate j (path-bit order)
    std::vector<Level> levels;        // levels[0] is the root (no crossing gate)
    HalfProgram half[2];              // 0 = A, 1 = B
    // pairs of path bits a path with a nonzero term sets equal (equal_bit_pairs); the others
    // are skipped
    std::vector<std::pair<int, int>> equal_bits;

    // tuning
    sf_tuning_t tuning{};
    // (half, first level, last level, p, R, dense)
    // (half, first, last, p, R, dense_m, prefix first, prefix last, prefix p) -> plan; prefix first
    // -1: no prefix (get_segment_plan_tail)
    std::map<std::tuple<int, int, int, int, int, int, int, int, int>, SegmentPlan> plan_cache;

    // device resources owned by the circuit
    void *dev_ws = nullptr;
    size_t dev_ws_bytes = 0;
    std::vector<void *> events;       // hipEvent_t pool of timed runs, reused across calls
    std::shared_ptr<void> exec_cache; // the last planned request (executor.cpp)
    int device_cus = 0;

    sf_run_stats_t stats{};
};

// planner.cpp
int build_programs(Circuit &c, std::string &err);
// Number of trailing tree levels folded into the gather with the current tuning (0 = none):
// the largest F for which both blocks' folds[F-1] qualify, capped by tuning.fold_levels.
int fold_depth(const Circuit &c);
// Pairs (u, v) of path bits with bit u == bit v in every path whose term is nonzero, and the
// test of one path id against them.
std::vector<std::pair<int, int>> equal_bit_pairs(const Circuit &c);
bool path_is_live(const Circuit &c, uint64_t id);
// Whether those FD levels use the general form (LeafFold::gen_ok) rather than the one whose
// non-diagonal gates act on branch qubits only.
bool fold_general(const Circuit &c, int FD);
// A level whose block-h operations are the projectors P_s of its crossing CZs (block A side),
// each the first operation on its qubit, followed only by one-qubit gates on the projected qubits:
// its node states are V P_s (parent state), V a tensor product of 2x2 matrices on those qubits,
// so the gather can read the parent's rows with the projected bits set to s and multiply by V's
// entry instead of reading states written for the level (the executor's deferred level).
constexpr int kMaxDeferredBits = 4;
struct DeferredLevel {
    bool ok = false;
    int n = 0;                                   // projected qubits (one path bit each)
    int q[kMaxDeferredBits] = {0};               // local qubit
    int u[kMaxDeferredBits] = {0};               // its path bit
    std::complex<double> v[kMaxDeferredBits][2][2];   // V_i[out][in], the unnormalised gates' product
    uint32_t mask = 0;                           // local qubits q[]
};
DeferredLevel deferred_level(const Circuit &c, int h, int level);
// dense_m: 0 = register/lane passes only; 2..4 = also fuse windows of up to dense_m qubits
// into dense 4-qubit blocks applied on matrix cores.
const SegmentPlan &get_segment_plan(Circuit &c, int half, int level, int p, int R, int dense_m = 0);
// The passes of the segments of levels first..last planned as one operation sequence (a chain
// of tree levels whose nodes have one child each run in the same slots, so their operations can
// share passes across the level boundaries).
const SegmentPlan &get_segment_plan_range(Circuit &c, int half, int first, int last, int p, int R, int dense_m = 0);
// The segment first..last with, in front of its operations, those of the last pass of the
// segment pre_first..pre_last planned for 2^pre_p slots (and that pass's rescaling): the plan of a
// fan-out whose parent level leaves its last pass to the children.  Passes of such a plan
// carry no known zero subspace.
const SegmentPlan &get_segment_plan_tail(Circuit &c, int half, int first, int last, int p, int R, int dense_m,
                                         int pre_first, int pre_last, int pre_p);

// sfpath.cpp: run_paths' argument checks and execution on a given workspace of any size (the
// entry point without allocations), and the thread's last_error() message.
int run_paths_in(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
                 const uint64_t *bitstrings, size_t n_bits, double *amps, uint32_t flags, void *hip_stream,
                 void *workspace, size_t workspace_bytes);
int set_error(int code, const std::string &msg);

// executor.cpp
// dry_run: plan the request (tree, batches, passes) and fill the launch and byte counts of
// c.stats without touching device memory.
int execute(Circuit &c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
            const uint64_t *bits, size_t n_bits, double *amps, uint32_t flags, void *stream,
            void *workspace, size_t workspace_bytes, std::string &err, bool dry_run = false,
            bool no_compile = false);
int estimate_workspace(const Circuit &c, uint64_t n_paths, size_t n_bits, uint32_t flags, size_t *bytes);

}  // namespace sf

// The C ABI's opaque circuit handle is the planner's circuit.
struct sf_circuit : sf::Circuit {};
