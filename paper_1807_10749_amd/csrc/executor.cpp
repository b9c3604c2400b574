// Executor: prefix tree of the requested paths, batches that fit the
// workspace, and the launch sequence (passes per tree level, fan-out
// copies with the branch operators, gather + FP64 path sum at the leaves).
//
// The paper keeps one checkpoint per process after the x_p-bit prefix and
// replays 2^x_b branches from it (Section 2); its logs show a second
// checkpoint level ("p + r + b").  Here every clock cycle that holds
// crossing gates is a tree level: the nodes of a level are the distinct
// prefixes of the requested path ids, a node's block states are evolved
// once and shared by all paths below it, and the states of many nodes of
// one level sit side by side as the slots of one batch array.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "jit.hpp"
#include "kernels.hpp"
#include "sf_host.hpp"

namespace sf {

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline uint64_t next_pow2(uint64_t x) { uint64_t p = 1; while (p < x) p <<= 1; return p; }
inline int log2u(uint64_t x) { int p = 0; while ((uint64_t(1) << p) < x) ++p; return p; }

struct Tree {
    std::vector<std::vector<uint64_t>> node;    // per level: path id of each node (bits below the level cleared)
    std::vector<std::vector<uint32_t>> parent;  // per level: index of the parent in the level above
    std::vector<std::vector<uint64_t>> first_child;  // per level: first child index, size |nodes|+1
};

int build_tree(const Circuit &c, const uint64_t *ids, uint64_t begin, uint64_t n, Tree &t, std::string &err)
{
    const int L = (int)c.levels.size() - 1;
    const int k = c.k;
    t.node.assign(L + 1, {});
    t.parent.assign(L + 1, {});
    t.first_child.assign(L + 1, {});
    std::vector<uint64_t> &leaf = t.node[L];     // the last level decides every path bit
    leaf.resize(n);
    if (ids) {
        std::copy(ids, ids + n, leaf.begin());
        std::sort(leaf.begin(), leaf.end());
        for (uint64_t i = 1; i < n; ++i)
            if (leaf[i] == leaf[i - 1]) { err = "path ids must be distinct"; return SF_ERR_INVALID; }
    } else {
        for (uint64_t i = 0; i < n; ++i) leaf[i] = begin + i;
    }
    if (n && (k < 64) && (leaf.back() >> k) != 0) { err = "path id >= 2^k"; return SF_ERR_INVALID; }
    // bottom-up: a level's nodes are the distinct prefixes of the level below (sorted input,
    // so equal prefixes are adjacent); the cost is the total node count, not leaves x levels
    for (int l = L - 1; l >= 0; --l) {
        const int drop = k - c.levels[l].bits_after;   // bits not yet decided at this level
        const std::vector<uint64_t> &below = t.node[l + 1];
        std::vector<uint64_t> &nd = t.node[l];
        std::vector<uint32_t> &par = t.parent[l + 1];
        par.resize(below.size());
        for (size_t i = 0; i < below.size(); ++i) {
            const uint64_t v = drop >= 64 ? 0 : ((below[i] >> drop) << drop);
            if (nd.empty() || nd.back() != v) nd.push_back(v);
            par[i] = (uint32_t)(nd.size() - 1);
        }
        std::vector<uint64_t> &fc = t.first_child[l];
        fc.assign(nd.size() + 1, 0);
        for (size_t i = 0; i < below.size(); ++i) fc[par[i] + 1]++;
        for (size_t i = 0; i < nd.size(); ++i) fc[i + 1] += fc[i];
    }
    return SF_OK;
}

struct LevelBuf {
    bool none = false;    // no buffer (leaf level folded into the gather)
    int alias = -1;       // level whose buffer this level reuses in place (chain levels)
    uint64_t cap = 1;     // slots
    size_t off[2] = {0, 0};
};

struct Launch {
    enum Kind { PASS, GATHER, DENSE, FOLD } kind;
    DenseArgs da{};
    FoldArgs fa{};
    FoldIswapArgs fia{};          // FOLD of crossing iSWAPs
    GFoldArgs gfa{};              // FOLD in the general form
    size_t mask_off = 0;          // FOLD: element offset of the batch's child masks
    bool defer = false;           // FOLD (general form): block A read from the parent batch (GFoldHalf)
    size_t dpar_off = 0, dsub_off = 0, dfac_off = 0;   // its per-slot tables (element offsets in tmaskv)
    int half = 0;
    int R = 0;
    bool flip = false;            // PASS: the program holds per-path flips
    bool pair_next = false;       // PASS: launched together with the next launch (the other block's pass)
    bool zskip = false;           // PASS: leaves the source's zero subspace unread (pa.n_zero entries)
    bool row_last = false;        // PASS: last pass of its block at the level the path sum reads
    PassArgs pa{};
    GatherArgs ga{};
    size_t plan_off = 0;      // device offset of the pass program inside the plan blob
    uint32_t prog_words = 0, groups_word = 0, terms_word = 0;
    int level = 0;
    size_t dst_off = 0, src_off = 0;   // buffer offsets inside the buffer region
    size_t table_off = 0;     // element offset of the batch's slot tables
    unsigned grid = 1;
    uint64_t bytes = 0;
    std::string jit_prog;         // PASS with tuning jit: its program as code (jit_program; "" = not covered)
    hipFunction_t jit_fn = nullptr;   // PASS: the compiled kernel of this pass (of the pair it heads)
};

struct BatchRec { int level; size_t table_off; uint64_t slots; };

// A segment's last pass left to the fan-out of its children: mask bit h = block h; the segment
// (levels first..last planned for 2^p slots) whose last pass the children's first pass applies.
struct Tail {
    int mask = 0;
    int first = 0, last = 0, p = 0;
};

// A run of PASS launches [begin, end) that executes as one chained launch (pass_chain_kernel).
struct ChainRec {
    size_t begin = 0, end = 0;
    uint32_t n_phases = 0;
    unsigned grid = 0;
    int R = 0;
    bool flip = false, zskip = false;
    size_t args_first = 0, phases_first = 0;   // entries in the call's chain argument arrays
};

// Grid of a chained launch of one kernel variant: at most one workgroup per compute unit, and at
// most half of what can be resident at once, so that chains launched on two streams fit side by
// side.  Cached per device.
unsigned chain_grid_limit(bool fp64, int R, bool flip, int cus)
{
    static std::mutex mu;
    static std::map<std::tuple<int, bool, int, bool>, unsigned> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    const auto key = std::make_tuple(dev, fp64, R, flip);
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    unsigned resident = 0;
    if (chain_max_grid(fp64, R, flip, chain_zskip(fp64, R, flip), &resident) != hipSuccess) resident = 0;
    const unsigned g = std::min<unsigned>((unsigned)std::max(cus, 0), resident / 2);
    cache[key] = g;
    return g;
}

struct BlobEntry { size_t off; uint32_t words, groups_word, terms_word; };

// Host-side result of planning one request: everything the enqueue step needs besides the
// device pointers of the call.
struct Planned {
    std::vector<LevelBuf> lb;
    size_t table_bound = 0;
    size_t rowmask_off = 0;               // row masks of both blocks, inside the table reservation
    uint64_t rowmask_words[2] = {0, 0};   // 32-bit words per block (0: no mask possible)
    std::vector<Launch> launches;
    std::vector<BatchRec> batches;
    std::vector<uint64_t> tpath;          // per slot of every batch: the node's path id
    std::vector<uint32_t> tparent;        // per slot: parent slot inside the parent batch
    std::vector<uint32_t> tmaskv;         // descendant masks of the batches the fold reads
    std::vector<char> blob;               // pass programs, dense matrices, fold tables
    size_t fold_tab_off[2] = {0, 0};
    size_t fold_off_off[2] = {0, 0};      // general fold: column offsets
    size_t plain_mask_idx = SIZE_MAX;
    uint64_t n_leaf_batches = 0;
};

// The circuit's last planned request; the next call reuses the plan if it is the same request
// (paths, bitstring count, layout flags, tuning, caller workspace).
struct ExecCache {
    bool valid = false;
    uint64_t n_paths = 0, path_begin = 0;
    size_t n_bits = 0;
    uint32_t flags = 0;
    bool has_ids = false;
    std::vector<uint64_t> ids;
    const void *ws = nullptr;
    size_t ws_bytes = 0;
    sf_tuning_t tuning{};
    int device_cus = 0;
    Planned plan;
};

}  // namespace

int estimate_workspace(const Circuit &c, uint64_t n_paths, size_t n_bits, uint32_t flags, size_t *bytes)
{
    const size_t elem = (flags & SF_FP64_SWEEPS) ? 16 : 8;
    const size_t sigma = (size_t(1) << c.half[0].q) * elem + (size_t(1) << c.half[1].q) * elem;
    const int L = (int)c.levels.size() - 1;
    const int FD = fold_depth(c);
    // upper bound: every level resident with min(2^bits, n_paths) nodes
    size_t total = 0;
    if (FD) total += align_up(n_paths * 8 + 64 * 8);   // descendant masks instead of folded levels
    for (int l = 0; l <= L; ++l) {
        if (l > L - FD) continue;
        const int b = c.levels[l].bits_after;
        uint64_t nodes = b >= 63 ? n_paths : std::min<uint64_t>(uint64_t(1) << b, n_paths);
        total += next_pow2(std::max<uint64_t>(nodes, 1)) * sigma;
        total += align_up(nodes * 12 + 64 * 12) ;
    }
    total += align_up(n_bits * 4) * 6 + align_up(n_bits * 8) + align_up(n_bits * 16) + (size_t(1) << 22);
    total += align_up(n_bits * 16) + (size_t(1) << 20);   // radix-sort scratch (bound)
    *bytes = total;
    return SF_OK;
}

int execute(Circuit &c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
            const uint64_t *bits, size_t n_bits, double *amps, uint32_t flags, void *stream_v,
            void *workspace, size_t workspace_bytes, std::string &err, bool dry_run, bool no_compile)
{
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t stream = (hipStream_t)stream_v;
    const bool fp64 = (flags & SF_FP64_SWEEPS) != 0;
    const bool plain = (flags & SF_PLAIN) != 0;
    const bool timing = (flags & SF_TIMING) != 0;
    const bool bits_dev = (flags & SF_BITS_ON_DEVICE) != 0;
    const bool out_dev = (flags & SF_OUT_ON_DEVICE) != 0;
    const size_t elem = fp64 ? 16 : 8;
    const int L = (int)c.levels.size() - 1;
    const int k = c.k;
    const int qh[2] = {c.half[0].q, c.half[1].q};
    int R = c.tuning.reg_qubits ? (int)c.tuning.reg_qubits : kMaxRegBits;
    R = std::max(1, std::min(R, fp64 ? kMaxRegBitsF64 : kMaxRegBits));
    int FD = fold_depth(c);                // trailing levels folded into the gather
    c.stats = sf_run_stats_t{};

    if (!path_ids && n_paths && k < 64 && ((path_begin + n_paths - 1) >> k) != 0) {
        err = "path range exceeds 2^k";
        return SF_ERR_INVALID;
    }
    if (path_ids)
        for (uint64_t i = 0; i < n_paths; ++i)
            if (k < 64 && (path_ids[i] >> k)) { err = "path id >= 2^k"; return SF_ERR_INVALID; }
    // paths whose term is zero (two projectors on one qubit decided by different path bits,
    // equal_bit_pairs) are dropped from the request; the rest run as an explicit list
    std::vector<uint64_t> live_ids;
    if (!c.equal_bits.empty() && n_paths) {
        bool all_live = true;
        for (uint64_t i = 0; i < n_paths && all_live; ++i)
            all_live = path_is_live(c, path_ids ? path_ids[i] : path_begin + i);
        if (!all_live) {
            live_ids.reserve(n_paths);
            for (uint64_t i = 0; i < n_paths; ++i) {
                const uint64_t id = path_ids ? path_ids[i] : path_begin + i;
                if (path_is_live(c, id)) live_ids.push_back(id);
            }
            path_ids = live_ids.data();
            path_begin = 0;
            n_paths = live_ids.size();
        }
    }
    c.stats.n_paths_live = n_paths;

    // The general fold reads 2^|S'| rows of the level above per bitstring and parent instead of
    // one row of each descendant: with the library choosing the depth (fold_levels 0) it is
    // used only when those reads are fewer bytes than writing the folded levels' states once
    // and gathering from them (a lower bound of that work), which holds when parents have many
    // requested descendants and fails for sparse path subsets.
    bool gfold = FD > 0 && fold_general(c, FD);
    if (gfold && !c.tuning.fold_levels && n_paths) {
        const LeafFold &a = c.half[0].folds[FD - 1], &b = c.half[1].folds[FD - 1];
        const int nbf = a.nb;
        uint64_t parents = n_paths;         // plain form: every path is its own tree
        if (plain) {
        } else if (!path_ids) {
            parents = ((path_begin + n_paths - 1) >> nbf) - (path_begin >> nbf) + 1;
        } else if (std::is_sorted(path_ids, path_ids + n_paths)) {
            parents = 1;
            for (uint64_t i = 1; i < n_paths; ++i) parents += (path_ids[i] >> nbf) != (path_ids[i - 1] >> nbf);
        }
        const double fold_b = (double)n_bits * (double)parents * (double)elem *
                              (std::ldexp(1.0, a.g_ns) + std::ldexp(1.0, b.g_ns));
        const double mat_b = (double)n_paths * (double)elem *
                                 (2.0 * FD * (std::ldexp(1.0, qh[0]) + std::ldexp(1.0, qh[1]))) +
                             (double)n_bits * (double)n_paths * 2.0 * (double)elem;
        if (fold_b >= mat_b) FD = 0;
    }
    const bool fold = FD > 0;
    gfold = gfold && fold;
    const int fold_at = L - FD;            // the level the gather reads
    const LeafFold *fh[2] = {fold ? &c.half[0].folds[FD - 1] : nullptr, fold ? &c.half[1].folds[FD - 1] : nullptr};
    // Deferred block-A level: when block A's operations at the level the general fold reads are
    // its crossing CZs' projectors and one-qubit gates on the projected qubits (deferred_level),
    // that level's block-A states are not written.  The fold reads the parent batch at the rows
    // whose projected bits equal the slot's path bits and multiplies by the gates' entry, which
    // saves the level's block-A writes (a fan-out of every parent into its children).
    DeferredLevel dA;
    bool defer = false;
    if (gfold && FD == 1 && fold_at >= 1 && !plain && !c.tuning.no_defer && n_paths) {
        dA = deferred_level(c, 0, fold_at);
        defer = dA.ok && !(dA.mask & fh[0]->g_smask);
    }
    const uint64_t all = c.n == 64 ? ~uint64_t(0) : ((uint64_t(1) << c.n) - 1);
    if (!bits_dev && !dry_run)
        for (size_t j = 0; j < n_bits; ++j)
            if (bits[j] & ~all) { err = "bitstring has bits outside the grid"; return SF_ERR_INVALID; }

    hipError_t he;
    if (!c.device_cus) {
        int dev = 0;
        if ((he = hipGetDevice(&dev)) != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(he); return SF_ERR_DEVICE; }
        if ((he = hipDeviceGetAttribute(&c.device_cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
            err = std::string("hipDeviceGetAttribute: ") + hipGetErrorString(he);
            return SF_ERR_DEVICE;
        }
    }

    // every block state needs at least 6 extended bits (one wave of lanes)
    const int qmin = std::min(qh[0], qh[1]);
    const uint64_t min_slots = qmin >= 6 ? 1 : (uint64_t(1) << (6 - qmin));
    const size_t sigma = (size_t(1) << qh[0]) * elem + (size_t(1) << qh[1]) * elem;   // bytes per slot, both blocks

    // ---------------------------------------------------------------- fixed workspace parts
    size_t fixed = 0;
    const size_t off_xa = fixed; fixed += align_up(n_bits * 4);
    const size_t off_xb = fixed; fixed += align_up(n_bits * 4);
    const size_t off_bits = fixed; if (!bits_dev) fixed += align_up(n_bits * 8);
    const size_t off_acc = fixed; if (!out_dev) fixed += align_up(n_bits * 16);
    const size_t off_flag = fixed; fixed += kAlign;
    // visiting order of the bitstrings, sorted by x_A on the device
    size_t sort_temp = 0;
    if ((he = sort_by_key_temp_bytes(std::max<uint64_t>(n_bits, 1), &sort_temp)) != hipSuccess) {
        err = std::string("sort temp size: ") + hipGetErrorString(he);
        return SF_ERR_DEVICE;
    }
    const size_t off_order = fixed; fixed += align_up(n_bits * 4);
    const size_t off_keys = fixed; fixed += align_up(n_bits * 4);
    const size_t off_idx = fixed; fixed += align_up(n_bits * 4);
    const size_t off_fkey = fixed; if (fold) fixed += align_up(n_bits * 4);
    const size_t off_sort_tmp = fixed; fixed += align_up(sort_temp);
    const size_t blob_budget = size_t(1) << 22;
    const size_t off_blob = fixed; fixed += blob_budget;
    // pass arguments and phase lists of the chained launches (runs that do not fit stay unchained)
    const size_t chain_budget = size_t(1) << 20;
    const size_t off_chain = fixed; fixed += chain_budget;

    auto dev_err = [&](const char *what, hipError_t e) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return SF_ERR_DEVICE;
    };
    // timed runs: event pairs from the circuit's pool (created on first use, reused by later
    // calls); pair i = pool entries 2i, 2i+1, bracketing a run of launches of one category
    std::vector<int> ev_cat;    // 0 sweep, 1 gather, 2 other
    auto ev_get = [&](size_t i) -> hipEvent_t {
        while (c.events.size() <= i) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            c.events.push_back((void *)e);
        }
        return (hipEvent_t)c.events[i];
    };
    auto ev_begin = [&](int cat) -> int {
        if (!timing) return -1;
        const int id = (int)ev_cat.size();
        hipEvent_t e = ev_get(2 * (size_t)id);
        if (!e || !ev_get(2 * (size_t)id + 1)) return -1;
        ev_cat.push_back(cat);
        (void)hipEventRecord(e, stream);
        return id;
    };
    auto ev_end = [&](int id) {
        if (id >= 0) (void)hipEventRecord((hipEvent_t)c.events[2 * (size_t)id + 1], stream);
    };

    // Bitstring preprocessing (upload, x_A / x_B, bad-bit flag, visiting order, group count).
    // It needs only the fixed part of the workspace, so with a caller's workspace it is enqueued
    // before the host plans the request and runs on the device meanwhile.
    bool pre_done = false;
    auto enqueue_pre = [&](char *wsp) -> int {
        pre_done = true;
        const uint64_t *d_bits = bits_dev ? bits : (const uint64_t *)(wsp + off_bits);
        int *d_flag = (int *)(wsp + off_flag);
        uint32_t *d_xa = (uint32_t *)(wsp + off_xa), *d_xb = (uint32_t *)(wsp + off_xb);
        const int id = ev_begin(2);
        if (!bits_dev && n_bits)
            if ((he = hipMemcpyAsync((void *)d_bits, bits, n_bits * 8, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy bitstrings", he);
        // flags: [0] bad bitstring, [1] visiting groups, [2] barrier fault of a chained launch,
        // [4..5] the chained launches' 64-bit barrier counter, [6..7] and [8..9] the set bits of
        // block A's and block B's row mask (64-bit)
        if ((he = launch_fill_zero_i32(d_flag, 10, stream)) != hipSuccess) return dev_err("fill", he);
        if ((he = launch_pext(d_bits, n_bits, c.mask_a, c.mask_b, all, d_xa, d_xb, d_flag, stream)) != hipSuccess) return dev_err("pext", he);
        const uint32_t *keys = d_xa;
        int key_bits = qh[0];
        if (fold) {
            // bitstrings that share their block-A bits outside the fold's S qubits read the same
            // rows of block A: visit them together
            const uint32_t kmask = (qh[0] >= 32 ? ~0u : ((1u << qh[0]) - 1)) &
                                   ~(gfold ? fh[0]->g_smask : fh[0]->iswap ? fh[0]->qmask : fh[0]->smask);
            if ((he = launch_key(d_xa, n_bits, kmask, (uint32_t *)(wsp + off_fkey), stream)) != hipSuccess) return dev_err("key", he);
            keys = (const uint32_t *)(wsp + off_fkey);
            key_bits = __builtin_popcount(kmask);
        }
        if ((he = launch_order_by_key(keys, (uint32_t *)(wsp + off_keys), (uint32_t *)(wsp + off_idx),
                                      (uint32_t *)(wsp + off_order), n_bits, key_bits, wsp + off_sort_tmp, sort_temp,
                                      stream)) != hipSuccess)
            return dev_err("sort", he);
        // groups of bitstrings that read the same block-A rows, for the byte accounting
        if ((he = launch_count_runs((const uint32_t *)(wsp + off_keys), n_bits, d_flag + 1, stream)) != hipSuccess)
            return dev_err("count", he);
        ev_end(id);
        return SF_OK;
    };
    if (workspace && !dry_run && workspace_bytes >= fixed) {
        const int rc = enqueue_pre((char *)workspace);
        if (rc) return rc;
    }

    // ---------------------------------------------------------------- tree and batch capacities
    // In plain form every path is its own one-node-per-level tree, run one after another.
    // A request identical to the circuit's previous one reuses its plan (launch list, slot
    // tables, programs); everything is still uploaded and enqueued.  Plain form rewrites its
    // tables per path and is planned every time.
    if (!c.exec_cache) c.exec_cache = std::make_shared<ExecCache>();
    ExecCache &cache = *static_cast<ExecCache *>(c.exec_cache.get());
    const uint32_t layout_flags = flags & ~uint32_t(SF_TIMING | SF_ACCUMULATE);
    const bool cacheable = n_paths && !plain && !dry_run && workspace;
    const bool hit = cacheable && cache.valid && cache.n_paths == n_paths && cache.n_bits == n_bits &&
                     cache.flags == layout_flags && cache.ws == workspace && cache.ws_bytes == workspace_bytes &&
                     cache.device_cus == c.device_cus && cache.has_ids == (path_ids != nullptr) &&
                     (path_ids ? std::equal(path_ids, path_ids + n_paths, cache.ids.begin())
                               : cache.path_begin == path_begin) &&
                     std::memcmp(&cache.tuning, &c.tuning, sizeof(sf_tuning_t)) == 0;
    Planned fresh;
    Planned &PL = hit ? cache.plan : fresh;
    std::vector<LevelBuf> &lb = PL.lb;
    size_t &table_bound = PL.table_bound;
    if (!hit) lb.assign(L + 1, LevelBuf());
    Tree tree;
    if (n_paths && !hit) {
        int rc;
        if (plain) {
            const uint64_t first = path_ids ? path_ids[0] : path_begin;
            if ((rc = build_tree(c, &first, 0, 1, tree, err))) return rc;
        } else if ((rc = build_tree(c, path_ids, path_begin, n_paths, tree, err))) {
            return rc;
        }
        for (int l = 1; l <= L; ++l)
            if (tree.node[l].size() == tree.node[l - 1].size()) lb[l].alias = lb[l - 1].alias >= 0 ? lb[l - 1].alias : l - 1;
        for (int l = fold_at + 1; fold && l <= L; ++l) { lb[l].none = true; lb[l].alias = -1; }
        const uint64_t maxs = c.tuning.max_slots ? c.tuning.max_slots : (uint64_t(1) << 20);
        const uint64_t leafmax = c.tuning.leaf_batch ? c.tuning.leaf_batch : maxs;
        for (int l = 0; l <= L; ++l) {
            uint64_t want = next_pow2(std::max<uint64_t>(tree.node[l].size(), 1));
            want = std::min(want, l == L ? leafmax : maxs);
            lb[l].cap = std::max(want, min_slots);
            // slot tables: at most twice the nodes (power-of-two padding), plus padding to
            // min_slots for at most one small batch per parent node, plus one padded batch
            table_bound += 2 * tree.node[l].size() + lb[l].cap + min_slots * (l ? tree.node[l - 1].size() : 1);
        }
        table_bound = align_up(table_bound * 8) + align_up(table_bound * 4);
        if (fold) table_bound += align_up(tree.node[fold_at].size() * 8 + 8);   // descendant masks
        // row masks of the last passes before the path sum: one bit per row of a block state
        PL.rowmask_off = table_bound;
        for (int h = 0; h < 2; ++h) {
            PL.rowmask_words[h] = (!c.tuning.no_row_skip && n_bits && qh[h] <= 30) ? ((uint64_t(1) << qh[h]) + 31) / 32 : 0;
            table_bound += align_up(PL.rowmask_words[h] * 4);
        }
        size_t budget;
        if (workspace) {
            if (workspace_bytes < fixed + table_bound) { err = "workspace too small"; return SF_ERR_OOM; }
            budget = workspace_bytes - fixed - table_bound;
        } else {
            size_t free_b = 0, total_b = 0;
            if ((he = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) return (err = std::string("hipMemGetInfo: ") + hipGetErrorString(he), SF_ERR_DEVICE);
            const size_t avail = c.dev_ws_bytes + (size_t)(0.85 * (double)free_b);
            if (avail < fixed + table_bound) { err = "not enough device memory"; return SF_ERR_OOM; }
            budget = avail - fixed - table_bound;
        }
        // shrink the largest owned level buffers until all fit
        for (;;) {
            for (int l = 1; l <= L; ++l) if (lb[l].alias >= 0) lb[l].cap = lb[lb[l].alias].cap;
            size_t need = 0;
            for (int l = 0; l <= L; ++l)
                if (lb[l].alias < 0 && !lb[l].none)
                    need += (defer && l == fold_at ? 0 : align_up(lb[l].cap * (size_t(1) << qh[0]) * elem)) +
                            align_up(lb[l].cap * (size_t(1) << qh[1]) * elem);
            if (need <= budget) break;
            int big = -1;
            for (int l = 0; l <= L; ++l)
                if (lb[l].alias < 0 && !lb[l].none && lb[l].cap > min_slots && (big < 0 || lb[l].cap >= lb[big].cap)) big = l;
            if (big < 0) { err = "workspace too small for one slot per tree level"; return SF_ERR_OOM; }
            lb[big].cap >>= 1;
        }
        size_t o = 0;
        for (int l = 0; l <= L; ++l) {
            if (lb[l].alias >= 0 || lb[l].none) continue;
            for (int h = 0; h < 2; ++h) {
                lb[l].off[h] = o;
                if (!(defer && l == fold_at && h == 0)) o += align_up(lb[l].cap * (size_t(1) << qh[h]) * elem);
            }
        }
        for (int l = 0; l <= L; ++l)
            if (lb[l].alias >= 0) { lb[l].off[0] = lb[lb[l].alias].off[0]; lb[l].off[1] = lb[lb[l].alias].off[1]; }
    }
    (void)sigma;

    // ---------------------------------------------------------------- launch list (depth first over batches)
    std::vector<Launch> &launches = PL.launches;
    std::vector<BatchRec> &batches = PL.batches;
    std::vector<uint64_t> &tpath = PL.tpath;
    std::vector<uint32_t> &tparent = PL.tparent;
    bool plan_error = false;
    std::vector<char> &blob = PL.blob;
    std::map<const SegmentPlan *, std::vector<BlobEntry>> blob_index;
    std::complex<double> leaf_scale[2];
    for (int h = 0; h < 2; ++h) {
        std::complex<double> s = c.half[h].init_scale;
        for (int l = 0; l <= L; ++l) s *= c.half[h].seg_scale[l];
        leaf_scale[h] = s;
    }
    const std::complex<double> gscale = leaf_scale[0] * leaf_scale[1];
    // folded levels are applied with their exact matrices, so their scalars are not tracked
    std::complex<double> fscale = 1.0;
    for (int h = 0; h < 2; ++h) {
        std::complex<double> s = c.half[h].init_scale;
        for (int l = 0; l <= fold_at; ++l) s *= c.half[h].seg_scale[l];
        fscale *= s;
    }
    std::vector<uint32_t> &tmaskv = PL.tmaskv;
    std::vector<uint64_t> node_mask;     // per node of the level the fold reads (filled below)
    size_t (&fold_tab_off)[2] = PL.fold_tab_off;
    size_t &plain_mask_idx = PL.plain_mask_idx;

    auto blob_entries = [&](const SegmentPlan &sp) -> const std::vector<BlobEntry> & {
        auto it = blob_index.find(&sp);
        if (it != blob_index.end()) return it->second;
        std::vector<BlobEntry> v;
        for (const PassPlan &pp : sp.passes) {
            if (pp.dense) {
                BlobEntry e{};
                e.off = align_up(blob.size());
                blob.resize(e.off + pp.mat.size() * sizeof(float));
                std::memcpy(blob.data() + e.off, pp.mat.data(), pp.mat.size() * sizeof(float));
                v.push_back(e);
                continue;
            }
            // [ops][pad to 8 bytes][groups][term bytes, padded to 4]
            std::vector<char> img(pp.ops.size() * sizeof(PassOp));
            if (!pp.ops.empty()) std::memcpy(img.data(), pp.ops.data(), img.size());
            while (img.size() % 8) img.push_back(0);
            BlobEntry e;
            e.groups_word = (uint32_t)(img.size() / 4);
            const size_t g0 = img.size();
            img.resize(g0 + pp.groups.size() * sizeof(DiagGroup));
            if (!pp.groups.empty()) std::memcpy(img.data() + g0, pp.groups.data(), pp.groups.size() * sizeof(DiagGroup));
            e.terms_word = (uint32_t)(img.size() / 4);
            img.insert(img.end(), pp.terms.begin(), pp.terms.end());
            while (img.size() % 4) img.push_back(0);
            e.words = (uint32_t)(img.size() / 4);
            if (e.words > (uint32_t)kMaxProgWords) plan_error = true;
            e.off = align_up(blob.size());
            blob.resize(e.off + img.size());
            std::memcpy(blob.data() + e.off, img.data(), img.size());
            v.push_back(e);
        }
        return blob_index.emplace(&sp, std::move(v)).first->second;
    };

    // gather byte accounting (see sf_run_stats_t): a_groups = distinct block-A keys of the visit
    auto account_gather = [&](const std::vector<Launch> &ls, uint64_t rounds, uint64_t a_groups) {
        c.stats.a_groups = a_groups;
        for (const Launch &ln : ls) {
            if (ln.kind != Launch::GATHER && ln.kind != Launch::FOLD) continue;
            const bool fi = ln.kind == Launch::FOLD && fh[0]->iswap;
            const uint64_t slots = ln.kind == Launch::FOLD ? (fi ? ln.fia.n_slots : gfold ? ln.gfa.n_slots : ln.fa.n_slots)
                                                           : ln.ga.n_slots;
            // parent rows per bitstring: 2^|S| (CZ form) or 2^G (iSWAP form) per block
            const uint64_t ra = ln.kind == Launch::FOLD ? uint64_t(1) << (fi ? fh[0]->ng : gfold ? fh[0]->g_ns : fh[0]->n_s) : 1;
            const uint64_t rb = ln.kind == Launch::FOLD ? uint64_t(1) << (fi ? fh[1]->ng : gfold ? fh[1]->g_ns : fh[1]->n_s) : 1;
            const uint64_t per = slots * elem * (a_groups * ra + (uint64_t)n_bits * rb) + (uint64_t)n_bits * 44 +
                                 (ln.kind == Launch::FOLD ? slots * 4 : 0);
            c.stats.n_gather_launches += rounds;
            c.stats.gather_ws_bytes = std::max<uint64_t>(c.stats.gather_ws_bytes, slots * (uint64_t(1) << qh[1]) * elem);
            c.stats.gather_bytes += rounds * per;
            c.stats.gather_row_bytes += rounds * ln.bytes;
        }
    };

    // grid cap of the sweep kernels: waves_per_cu / 4 workgroups per compute unit (default 128
    // waves, more than can be resident: short workgroups keep every channel busy to the end)
    const unsigned max_grid = (unsigned)std::max(1, c.device_cus) * (c.tuning.waves_per_cu ? std::max(1u, c.tuning.waves_per_cu / 4) : 32);
    uint64_t &n_leaf_batches = PL.n_leaf_batches;
    // the batch that a deferred level's fold reads block A from: its offset, slot bits, and the
    // parent slot of each slot of the batch being visited
    size_t defer_par_off = 0;
    int defer_par_p = 0;
    std::vector<uint32_t> defer_par;

    // appends the slot tables of one batch (padded to `slots` entries)
    auto put_tables = [&](const std::vector<uint64_t> &paths, const std::vector<uint32_t> &parents, uint64_t slots) {
        const size_t off = tpath.size();
        for (uint64_t i = 0; i < slots; ++i) {
            const size_t j = std::min<size_t>(i, paths.size() - 1);
            tpath.push_back(paths[j]);
            tparent.push_back(parents[j]);
        }
        return off;
    };

    // n_real: slots in use (the rest of the nslots pad the batch to a power of two); src_read:
    // parent slots a fan-out actually reads (distinct parents of its children), for the byte
    // count, 0 = all src_slots
    // level0 < level: the segments of levels level0..level as one (chain levels, chain_run).
    // drop: bit h = block h leaves its segment's last pass to the fan-out of the children
    // (tail_moves); pre: the parent segment whose dropped last pass this fan-out applies first.
    auto add_segment = [&](int level, uint64_t nslots, uint64_t n_real, const size_t dst[2], int mode,
                           const size_t src[2], uint64_t src_slots, size_t table_off, int n_low = 0,
                           int low_first = 0, uint64_t src_read = 0, int level0 = -1, int drop = 0,
                           const Tail *pre = nullptr) {
        const int lev0 = level0 < 0 ? level : level0;
        const int p = log2u(nslots);
        const uint64_t slots_real = n_real && n_real < nslots ? n_real : 0;
        const uint64_t used = slots_real ? slots_real : nslots;
        const int ps = log2u(src_slots);
        std::vector<Launch> hl[2];      // each block's launches of this segment, in order
        for (int h = 0; h < 2; ++h) {
            if (defer && h == 0 && level == fold_at) continue;   // block A's states of this level are not written
            const int dm = fp64 ? 0 : (int)c.tuning.dense_qubits;
            const SegmentPlan &sp = pre && ((pre->mask >> h) & 1)
                                        ? get_segment_plan_tail(c, h, lev0, level, p, R, dm, pre->first, pre->last, pre->p)
                                        : get_segment_plan_range(c, h, lev0, level, p, R, dm);
            if (!sp.ok) { plan_error = true; return; }
            const std::vector<BlobEntry> &be = blob_entries(sp);
            const int n_ext = p + qh[h];
            const size_t n_pass = sp.passes.size() - (((drop >> h) & 1) ? 1 : 0);
            for (size_t i = 0; i < n_pass; ++i) {
                const PassPlan &pp = sp.passes[i];
                if (pp.dense) {
                    Launch ln;
                    ln.kind = Launch::DENSE;
                    ln.half = h;
                    ln.level = level;
                    std::memset(&ln.da, 0, sizeof(ln.da));
                    ln.da.n_groups = uint64_t(1) << (n_ext - 9);
                    ln.da.rescale = std::ldexp(1.0, -pp.rescale_exp);
                    ln.da.p = p;
                    ln.da.slots_real = slots_real;
                    for (int t = 0; t < 4; ++t) ln.da.bpos[t] = pp.bpos[t];
                    ln.dst_off = dst[h];
                    ln.src_off = dst[h];
                    ln.plan_off = be[i].off;
                    ln.grid = (unsigned)std::min<uint64_t>((ln.da.n_groups + 3) / 4, max_grid);
                    ln.bytes = used * (uint64_t(1) << qh[h]) * elem * 2;
                    hl[h].push_back(ln);
                    continue;
                }
                Launch ln;
                ln.kind = Launch::PASS;
                ln.half = h;
                ln.R = pp.R;
                ln.flip = pp.has_flip;
                ln.level = level;
                PassArgs &a = ln.pa;
                std::memset(&a, 0, sizeof(a));
                a.n_tiles = uint64_t(1) << (n_ext - 6 - pp.R);
                a.n_ops = (uint32_t)pp.ops.size();
                a.p_dst = p;
                a.p_src = p;
                a.src_mode = SRC_SAME;
                a.rescale = std::ldexp(1.0, -pp.rescale_exp);
                a.slots_real = slots_real;
                for (int kk = 0; kk < 6; ++kk) a.reg_pos[kk] = pp.reg_pos[kk];
                a.lane_qpos = pp.lane_q >= 0 ? p + pp.lane_q : 0;
                a.lane_qpos4 = pp.lane_q >= 0 && pp.lane_q4 >= 0 ? p + pp.lane_q4 : 0;
                {
                    // sibling bits as the lowest tile bits (first pass of a regular fan-out only)
                    std::vector<int> skip(pp.reg_pos, pp.reg_pos + pp.R);
                    if (pp.lane_q >= 0) skip.push_back(p + pp.lane_q);
                    if (pp.lane_q >= 0 && pp.lane_q4 >= 0) skip.push_back(p + pp.lane_q4);
                    a.n_low = 0;
                    if (i == 0 && mode == SRC_FANOUT && n_low > 0)
                        for (int t = 0; t < n_low; ++t) {
                            a.low_pos[a.n_low++] = low_first + t;
                            skip.push_back(low_first + t);
                        }
                    std::sort(skip.begin(), skip.end());
                    a.n_skip = (int)skip.size();
                    for (size_t t = 0; t < skip.size(); ++t) a.skip_pos[t] = skip[t];
                }
                if (c.tuning.jit) ln.jit_prog = jit_program(pp);
                ln.dst_off = dst[h];
                ln.src_off = dst[h];
                if (i == 0 && mode == SRC_INIT) {
                    a.src_mode = SRC_INIT;
                    uint64_t z = 0;
                    for (int t = 0; t < qh[h]; ++t)
                        if (!((c.half[h].init_h_mask >> t) & 1)) z |= uint64_t(1) << (p + t);
                    a.init_zero_mask = z;
                } else if (i == 0 && mode == SRC_FANOUT) {
                    a.src_mode = SRC_FANOUT;
                    a.p_src = ps;
                    ln.src_off = src[h];
                }
                // zero subspace of the source (the initial state has none): its amplitudes are
                // left unread, and the algorithmic bytes count the reads of the rest (at most
                // 2^-|qubits| of the state; two entries on one qubit can zero whole slots)
                int z_qubits = 0;
                a.n_zero = 0;
                if (a.src_mode != SRC_INIT) {
                    uint64_t zq = 0;
                    for (const auto &e : pp.zero_in) {
                        if (a.n_zero == kMaxZeroEntries) break;
                        const int pos_e = p + e.first;
                        int r = -1;
                        for (int kk = 0; kk < pp.R; ++kk)
                            if (pp.reg_pos[kk] == pos_e) r = kk;
                        a.zero_reg[a.n_zero] = (int8_t)r;
                        a.zero_pos[a.n_zero] = (uint8_t)pos_e;
                        a.zero_bit[a.n_zero] = e.second;
                        ++a.n_zero;
                        zq |= uint64_t(1) << e.first;
                    }
                    z_qubits = __builtin_popcountll(zq);
                }
                ln.zskip = a.n_zero > 0 && !fp64 && !pp.has_flip && (pp.R == 4 || pp.R == 5);
                if (!ln.zskip) {
                    a.n_zero = 0;
                    z_qubits = 0;
                }
                ln.table_off = table_off;
                ln.plan_off = be[i].off;
                ln.prog_words = be[i].words;
                ln.groups_word = be[i].groups_word;
                ln.terms_word = be[i].terms_word;
                ln.grid = (unsigned)std::min<uint64_t>((a.n_tiles + 3) / 4, max_grid);
                // algorithmic bytes over the slots in use: the state written once, the source read
                // once (its non-zero part)
                const uint64_t state_bytes = used * (uint64_t(1) << qh[h]) * elem;
                ln.bytes = state_bytes;
                if (a.src_mode == SRC_SAME) ln.bytes += state_bytes >> z_qubits;
                if (a.src_mode == SRC_FANOUT)
                    ln.bytes += (src_read ? src_read : uint64_t(1) << ps) * (uint64_t(1) << qh[h]) * elem >> z_qubits;
                hl[h].push_back(ln);
            }
        }
        // the last pass of each block at the level the path sum reads may skip the tiles no
        // requested bitstring reads (row masks, decided once the plan is complete)
        if (level == fold_at)
            for (int h = 0; h < 2; ++h)
                if (!hl[h].empty() && hl[h].back().kind == Launch::PASS) hl[h].back().row_last = true;
        // The two blocks' passes are independent: interleave them, and launch the i-th pass of
        // block A together with the i-th pass of block B (one kernel, the blocks of the grid split
        // between them) when both run the same kernel variant.  Small levels are bound by launch
        // and wave latency, which the pair then pays once.
        for (size_t i = 0; i < std::max(hl[0].size(), hl[1].size()); ++i) {
            const bool both = i < hl[0].size() && i < hl[1].size();
            if (i < hl[0].size()) {
                Launch ln = hl[0][i];
                ln.pair_next = both && ln.kind == Launch::PASS && hl[1][i].kind == Launch::PASS &&
                               ln.R == hl[1][i].R && ln.flip == hl[1][i].flip;
                launches.push_back(ln);
            }
            if (i < hl[1].size()) launches.push_back(hl[1][i]);
        }
    };

    // Chain levels: below level l every node has one child, evolved in place in the same slots.
    // Returns the deepest level last such that levels l+1..last are all chain levels (stopping
    // before a deferred level), with nodes[] advanced to it; the segments of levels first..last
    // then run as one plan when that takes no more passes than planning them one by one.
    auto chain_run = [&](int l, std::vector<uint32_t> &nodes) {
        int last = l;
        while (last + 1 <= L && lb[last + 1].alias >= 0 && !(defer && last + 1 == fold_at)) {
            const std::vector<uint64_t> &fc = tree.first_child[last];
            for (uint32_t &x : nodes) x = (uint32_t)fc[x];
            ++last;
        }
        return last;
    };
    auto merge_ok = [&](int first, int last, uint64_t nslots) {
        if (first == last) return true;
        if (c.tuning.no_chain_merge) return false;
        const int p = log2u(nslots), dm = fp64 ? 0 : (int)c.tuning.dense_qubits;
        size_t merged = 0, apart = 0;
        for (int h = 0; h < 2; ++h) {
            const SegmentPlan &m = get_segment_plan_range(c, h, first, last, p, R, dm);
            if (!m.ok) return false;
            merged += m.passes.size();
            for (int lv = first; lv <= last; ++lv) apart += get_segment_plan(c, h, lv, p, R, dm).passes.size();
        }
        return merged <= apart;
    };

    // Whether each block's segment first..last (the batch `nodes` of 2^p slots at level last)
    // leaves its last pass to the fan-out of its children, which then apply that pass's
    // operations first: it saves reading and writing the parent batch once, for running those
    // operations once per child.  Taken when the children are written by a fan-out (level
    // last + 1 is not a chain level, not folded into the path sum, not block A's deferred level),
    // the segment's last pass is an in-place pass that is not a dense block, the parents have at
    // most 16 children each, and the children's plan with those operations takes no more passes
    // than without (tuning no_tail_move = 1: never).  keep: blocks whose segment here itself
    // starts with its parent's last pass (their plan is not the one the children would take the
    // last pass of), which keep theirs.
    auto tail_moves = [&](int first, int last, const std::vector<uint32_t> &nodes, uint64_t nslots, int keep = 0) {
        Tail t;
        t.first = first;
        t.last = last;
        t.p = log2u(nslots);
        if (c.tuning.no_tail_move || nodes.empty() || last + 1 > L || lb[last + 1].alias >= 0 || lb[last + 1].none ||
            (fold && last == fold_at))
            return t;
        const std::vector<uint64_t> &fc = tree.first_child[last];
        uint64_t nch = 0;
        for (uint32_t x : nodes) nch += fc[x + 1] - fc[x];
        if (nch > 16 * (uint64_t)nodes.size()) return t;
        const uint64_t cs = std::max<uint64_t>(std::min<uint64_t>(next_pow2(nch), lb[last + 1].cap), min_slots);
        const int pc = log2u(cs);
        const int dm = fp64 ? 0 : (int)c.tuning.dense_qubits;
        for (int h = 0; h < 2; ++h) {
            if ((keep >> h) & 1) continue;
            if (defer && h == 0 && last + 1 == fold_at) continue;   // the fold reads this batch as it is
            const SegmentPlan &par = get_segment_plan_range(c, h, first, last, t.p, R, dm);
            if (!par.ok || par.passes.size() < 2 || par.passes.back().dense) continue;
            const SegmentPlan &with = get_segment_plan_tail(c, h, last + 1, last + 1, pc, R, dm, first, last, t.p);
            const SegmentPlan &without = get_segment_plan_range(c, h, last + 1, last + 1, pc, R, dm);
            if (with.ok && without.ok && with.passes.size() <= without.passes.size()) t.mask |= 1 << h;
        }
        return t;
    };

    // nodes: node indices of this batch in slot order; pre: this batch's segment's last pass, left
    // to the children (tail_moves)
    std::function<void(int, const std::vector<uint32_t> &, uint64_t, const Tail &)> visit;
    visit = [&](int l, const std::vector<uint32_t> &nodes, uint64_t nslots, const Tail &pre) {
        if (plan_error) return;
        const int own = lb[l].alias >= 0 ? lb[l].alias : l;
        if (fold && l == fold_at) {
            // the gather reads this batch and applies the folded levels itself
            Launch ln;
            ln.kind = Launch::FOLD;
            ln.level = l;
            const int nd = 1 << fh[0]->nb;                       // descendants per node (one mask bit each)
            const uint64_t full = nd >= 64 ? ~uint64_t(0) : (uint64_t(1) << nd) - 1;
            bool all = true;
            for (size_t i = 0; i < nodes.size(); ++i) all = all && node_mask[nodes[i]] == full;
            if (fh[0]->iswap) {
                FoldIswapArgs &f = ln.fia;
                std::memset(&f, 0, sizeof(f));
                for (int h = 0; h < 2; ++h) {
                    const LeafFold &lf = *fh[h];
                    FoldIswapHalf &d = f.h[h];
                    d.qmask = lf.qmask;
                    d.tmask = lf.tmask;
                    d.n_s = lf.n_s;
                    for (int g = 0; g < lf.ng; ++g) {
                        d.q[g] = (uint8_t)lf.gq[g];
                        d.ypos[g] = (int8_t)lf.gy[g];
                    }
                }
                for (int g = 0; g < fh[0]->ng; ++g) f.u[g] = (uint8_t)fh[0]->gu[g];
                f.n_bits = n_bits;
                f.n_slots = (uint32_t)nodes.size();
                f.p = log2u(nslots);
                f.scale_re = fscale.real();
                f.scale_im = fscale.imag();
                f.all_children = all && !plain ? 1 : 0;
                // 64-bit masks, two words each (the first one 8-byte aligned)
                if (tmaskv.size() & 1) tmaskv.push_back(0);
                ln.mask_off = tmaskv.size();
                if (plain) plain_mask_idx = tmaskv.size();
                for (size_t i = 0; i < nodes.size(); ++i) {
                    tmaskv.push_back((uint32_t)node_mask[nodes[i]]);
                    tmaskv.push_back((uint32_t)(node_mask[nodes[i]] >> 32));
                }
                ln.bytes = (uint64_t)n_bits * (uint64_t)nodes.size() * elem * (uint64_t(2) << fh[0]->ng);
            } else if (gfold) {
                GFoldArgs &f = ln.gfa;
                std::memset(&f, 0, sizeof(f));
                for (int h = 0; h < 2; ++h) {
                    const LeafFold &lf = *fh[h];
                    f.h[h].smask = lf.g_smask;
                    f.h[h].tmask = lf.g_tmask;
                    f.h[h].n_s = lf.g_ns;
                    f.h[h].n_rest = lf.g_ns - lf.nb;
                }
                f.n_bits = n_bits;
                f.n_slots = (uint32_t)nodes.size();
                f.p = log2u(nslots);
                f.scale_re = fscale.real();
                f.scale_im = fscale.imag();
                ln.mask_off = tmaskv.size();
                if (plain) plain_mask_idx = tmaskv.size();
                for (size_t i = 0; i < nodes.size(); ++i) tmaskv.push_back((uint32_t)node_mask[nodes[i]]);
                f.all_children = all && !plain ? 1 : 0;
                ln.bytes = (uint64_t)n_bits * (uint64_t)nodes.size() * elem *
                           ((uint64_t(1) << fh[0]->g_ns) + (uint64_t(1) << fh[1]->g_ns));
                if (defer) {
                    // block A from the parent batch: per slot its parent slot, the projected bits
                    // (the slot's path bits at the projected qubits) and the deferred gates'
                    // entries V[x at the projected qubits][path bits] (with the segment's power of
                    // two that its passes would have divided out)
                    ln.defer = true;
                    f.h[0].p_par = defer_par_p;
                    f.h[0].dmask = dA.mask;
                    f.h[0].nd = dA.n;
                    ln.dst_off = defer_par_off;
                    ln.dpar_off = tmaskv.size();
                    for (size_t i = 0; i < nodes.size(); ++i) tmaskv.push_back(defer_par[i]);
                    ln.dsub_off = tmaskv.size();
                    const std::vector<uint64_t> &pid = tree.node[fold_at];
                    for (size_t i = 0; i < nodes.size(); ++i) {
                        uint32_t sub = 0;
                        for (int k = 0; k < dA.n; ++k) sub |= (uint32_t)((pid[nodes[i]] >> dA.u[k]) & 1u) << dA.q[k];
                        tmaskv.push_back(sub);
                    }
                    while (tmaskv.size() & 3) tmaskv.push_back(0);   // 16-byte aligned complex entries
                    ln.dfac_off = tmaskv.size();
                    const double e2 = std::ldexp(1.0, -c.half[0].seg_rescale_exp[fold_at]);
                    int rank[kMaxDeferredBits];
                    for (int k = 0; k < dA.n; ++k) rank[k] = __builtin_popcount(dA.mask & ((1u << dA.q[k]) - 1u));
                    for (size_t i = 0; i < nodes.size(); ++i)
                        for (uint32_t xd = 0; xd < (1u << dA.n); ++xd) {
                            std::complex<double> v = e2;
                            for (int k = 0; k < dA.n; ++k)
                                v *= dA.v[k][(xd >> rank[k]) & 1u][(pid[nodes[i]] >> dA.u[k]) & 1u];
                            if (fp64) {
                                uint32_t w[4];
                                const double d2[2] = {v.real(), v.imag()};
                                std::memcpy(w, d2, 16);
                                tmaskv.insert(tmaskv.end(), w, w + 4);
                            } else {
                                uint32_t w[2];
                                const float f2[2] = {(float)v.real(), (float)v.imag()};
                                std::memcpy(w, f2, 8);
                                tmaskv.insert(tmaskv.end(), w, w + 2);
                            }
                        }
                }
            } else {
                FoldArgs &f = ln.fa;
                std::memset(&f, 0, sizeof(f));
                for (int h = 0; h < 2; ++h) {
                    const LeafFold &lf = *fh[h];
                    FoldHalf &d = f.h[h];
                    d.smask = lf.smask;
                    d.tmask = lf.tmask;
                    d.n_s = lf.n_s;
                    d.dsel = 0;
                    for (int u = 0; u < lf.nb; ++u) {
                        d.bq[u] = (uint8_t)lf.bq[u];
                        if (lf.ypos[u] >= 0) {
                            d.sstride[u] = 1u << lf.bq[u];
                            d.ypos[u] = (uint8_t)lf.ypos[u];
                        } else {
                            d.dsel |= 1u << u;
                        }
                    }
                }
                f.n_bits = n_bits;
                f.n_slots = (uint32_t)nodes.size();
                f.p = log2u(nslots);
                f.scale_re = fscale.real();
                f.scale_im = fscale.imag();
                ln.mask_off = tmaskv.size();
                if (plain) plain_mask_idx = tmaskv.size();
                for (size_t i = 0; i < nodes.size(); ++i) tmaskv.push_back((uint32_t)node_mask[nodes[i]]);
                f.all_children = all && !plain ? 1 : 0;
                ln.bytes = (uint64_t)n_bits * (uint64_t)nodes.size() * elem *
                           ((uint64_t(1) << fh[0]->n_s) + (uint64_t(1) << fh[1]->n_s));
            }
            if (!ln.defer) ln.dst_off = lb[own].off[0];
            ln.src_off = lb[own].off[1];
            launches.push_back(ln);
            ++n_leaf_batches;
            return;
        }
        if (l == L) {
            Launch ln;
            ln.kind = Launch::GATHER;
            ln.level = l;
            GatherArgs &g = ln.ga;
            std::memset(&g, 0, sizeof(g));
            g.n_bits = n_bits;
            g.n_slots = (uint32_t)nodes.size();
            g.p = log2u(nslots);
            g.scale_re = gscale.real();
            g.scale_im = gscale.imag();
            ln.dst_off = lb[own].off[0];
            ln.src_off = lb[own].off[1];
            ln.bytes = (uint64_t)n_bits * (uint64_t)nodes.size() * 2 * elem;
            launches.push_back(ln);
            ++n_leaf_batches;
            return;
        }
        const std::vector<uint64_t> &fc = tree.first_child[l];
        const std::vector<uint64_t> &cnode = tree.node[l + 1];
        if (lb[l + 1].alias >= 0) {
            // chain level(s): one child per node, evolved in place in the same slots; a run of
            // them is planned as one segment when that saves passes
            std::vector<uint32_t> ch(nodes.size());
            for (size_t i = 0; i < nodes.size(); ++i) ch[i] = (uint32_t)fc[nodes[i]];
            std::vector<uint32_t> deep(ch);
            int last = chain_run(l + 1, deep);
            if (!merge_ok(l + 1, last, nslots)) last = l + 1;
            else ch.swap(deep);
            std::vector<uint64_t> pv(nodes.size());
            std::vector<uint32_t> pz(nodes.size(), 0);
            for (size_t i = 0; i < nodes.size(); ++i) pv[i] = tree.node[last][ch[i]];
            const size_t toff = put_tables(pv, pz, nslots);
            batches.push_back(BatchRec{last, toff, nslots});
            const size_t base[2] = {lb[own].off[0], lb[own].off[1]};
            // (a level above a chain level keeps its last pass: tail_moves wants a fan-out)
            const Tail tl = tail_moves(l + 1, last, ch, nslots);
            add_segment(last, nslots, nodes.size(), base, SRC_SAME, base, nslots, toff, 0, 0, 0, l + 1, tl.mask);
            if (defer && last == fold_at) {
                // in place: block A's slots still hold the parents' states
                defer_par_off = base[0];
                defer_par_p = log2u(nslots);
                defer_par.resize(nodes.size());
                for (size_t i = 0; i < nodes.size(); ++i) defer_par[i] = (uint32_t)i;
            }
            visit(last, ch, nslots, tl);
            return;
        }
        // Slot order of the children.  Full fan-outs (every parent has all 2^n_cut children) go
        // branch-major, (new path bits of the child, parent slot), so that consecutive slots of
        // one branch value read consecutive parent slots.  Otherwise, with m children per parent,
        // one branch value holds only a fraction m / 2^n_cut of the parents: a wave's parent
        // reads would skip the parents without that child, and every parent would be fetched
        // once per child.  Parent-major order (the order the children are collected in) makes
        // the reads contiguous instead, with m lanes on each parent value, so each parent is
        // fetched about once.
        const int shift = k - c.levels[l + 1].bits_after;
        const uint64_t bmask = (uint64_t(1) << c.levels[l + 1].n_cut) - 1;
        struct Ch { uint64_t b; uint32_t slot; uint32_t node; };
        std::vector<Ch> chs;
        for (size_t i = 0; i < nodes.size(); ++i)
            for (uint64_t cc = fc[nodes[i]]; cc < fc[nodes[i] + 1]; ++cc)
                chs.push_back(Ch{shift >= 64 ? 0 : ((cnode[cc] >> shift) & bmask), (uint32_t)i, (uint32_t)cc});
        if (chs.size() == nodes.size() << c.levels[l + 1].n_cut)
            std::stable_sort(chs.begin(), chs.end(),
                             [](const Ch &x, const Ch &y) { return x.b != y.b ? x.b < y.b : x.slot < y.slot; });
        const LevelBuf &cb = lb[l + 1];
        const size_t src[2] = {lb[own].off[0], lb[own].off[1]};
        // regular fan-out: every parent slot has all 2^n_cut children and the parent batch is
        // unpadded, so chunk slot = (branch value - first) * nslots + parent slot
        const bool regular = nodes.size() == nslots && nslots >= 64 &&
                             chs.size() == nodes.size() << c.levels[l + 1].n_cut;
        for (size_t a0 = 0; a0 < chs.size(); a0 += cb.cap) {
            const size_t a1 = std::min(chs.size(), a0 + (size_t)cb.cap);
            const uint64_t ns = std::max<uint64_t>(next_pow2(a1 - a0), min_slots);
            int n_low = 0;
            if (regular && (a1 - a0) % nslots == 0 && a0 % nslots == 0) {
                const uint64_t sib = (a1 - a0) / nslots;           // branch values in this chunk
                if ((sib & (sib - 1)) == 0) n_low = std::min(3, log2u(sib));
            }
            std::vector<uint32_t> ch(a1 - a0), par(a1 - a0);
            std::vector<uint64_t> pv(a1 - a0);
            for (size_t i = a0; i < a1; ++i) { ch[i - a0] = chs[i].node; par[i - a0] = chs[i].slot; pv[i - a0] = cnode[chs[i].node]; }
            // distinct parents read by this chunk (each parent's children are adjacent in
            // parent-major order; in branch-major order a chunk spans whole runs of parents)
            uint64_t n_read = 0;
            {
                std::vector<uint32_t> u(par);
                std::sort(u.begin(), u.end());
                n_read = (uint64_t)(std::unique(u.begin(), u.end()) - u.begin());
            }
            const size_t toff = put_tables(pv, par, ns);
            batches.push_back(BatchRec{l + 1, toff, ns});
            const size_t dst[2] = {cb.off[0], cb.off[1]};
            const Tail tl = tail_moves(l + 1, l + 1, ch, ns, pre.mask);
            add_segment(l + 1, ns, a1 - a0, dst, SRC_FANOUT, src, nslots, toff, n_low, log2u(nslots), n_read, -1,
                        tl.mask, &pre);
            if (defer && l + 1 == fold_at) {
                defer_par_off = src[0];
                defer_par_p = log2u(nslots);
                defer_par = par;
            }
            visit(l + 1, ch, ns, tl);
            if (plan_error) return;
        }
    };

    // per node of the level the gather reads: bit i set if its descendant with branch value i
    // (the low path bits decided by the folded levels) is requested
    if (n_paths && fold && !hit) {
        node_mask.assign(tree.node[fold_at].size(), 0);
        const uint64_t low = (uint64_t(1) << fh[0]->nb) - 1;
        for (size_t i = 0; i < tree.node[L].size(); ++i) {
            size_t a = i;
            for (int l = L; l > fold_at; --l) a = tree.parent[l][a];
            node_mask[a] |= uint64_t(1) << (tree.node[L][i] & low);
        }
    }
    if (n_paths && gfold && !hit) {
        // general fold: the table in the state precision and the column offsets
        for (int h = 0; h < 2; ++h) {
            const std::vector<std::complex<double>> &tab = fh[h]->gtab;
            fold_tab_off[h] = align_up(blob.size());
            blob.resize(fold_tab_off[h] + tab.size() * elem);
            for (size_t i = 0; i < tab.size(); ++i) {
                if (fp64) {
                    const double v[2] = {tab[i].real(), tab[i].imag()};
                    std::memcpy(blob.data() + fold_tab_off[h] + 16 * i, v, 16);
                } else {
                    const float v[2] = {(float)tab[i].real(), (float)tab[i].imag()};
                    std::memcpy(blob.data() + fold_tab_off[h] + 8 * i, v, 8);
                }
            }
            const std::vector<uint32_t> &off = fh[h]->goff;
            PL.fold_off_off[h] = align_up(blob.size());
            blob.resize(PL.fold_off_off[h] + off.size() * 4);
            std::memcpy(blob.data() + PL.fold_off_off[h], off.data(), off.size() * 4);
        }
    } else if (n_paths && fold && !hit) {
        for (int h = 0; h < 2; ++h) {
            const std::vector<std::complex<double>> &tab = fh[h]->tab;
            fold_tab_off[h] = align_up(blob.size());
            blob.resize(fold_tab_off[h] + tab.size() * 16);
            for (size_t i = 0; i < tab.size(); ++i) {
                const double v[2] = {tab[i].real(), tab[i].imag()};
                std::memcpy(blob.data() + fold_tab_off[h] + 16 * i, v, 16);
            }
        }
    }
    if (n_paths && !hit) {
        const uint64_t ns0 = std::max<uint64_t>(1, min_slots);
        // the root and the chain levels below it (one node each) as one segment when that saves passes
        std::vector<uint32_t> deep{0};
        int last = chain_run(0, deep);
        if (!merge_ok(0, last, ns0)) {
            last = 0;
            deep.assign(1, 0);
        }
        const size_t toff = put_tables(std::vector<uint64_t>{tree.node[last][deep[0]]}, std::vector<uint32_t>{0}, ns0);
        batches.push_back(BatchRec{last, toff, ns0});
        const size_t base0[2] = {lb[0].off[0], lb[0].off[1]};
        const Tail tl = tail_moves(0, last, deep, ns0);
        add_segment(last, ns0, 1, base0, SRC_INIT, base0, ns0, toff, 0, 0, 0, 0, tl.mask);
        visit(last, deep, ns0, tl);
    }
    if (plan_error) { err = "internal: a segment could not be scheduled into passes"; return SF_ERR_UNSUPPORTED; }
    if (blob.size() > blob_budget) { err = "internal: pass programs exceed their reservation"; return SF_ERR_UNSUPPORTED; }
    const size_t tables_bytes = align_up(tpath.size() * 8) + align_up(tparent.size() * 4) + align_up(tmaskv.size() * 4);

    // Chains (tuning chain_passes): maximal runs of consecutive PASS launches (a pair is one
    // phase) of one kernel variant whose grids are at most chain_grid_limit run as one cooperative
    // launch with a grid barrier between phases: one launch per run of small tree levels instead
    // of one per pass.  On MI355X a grid barrier of 256 workgroups (one device-scope atomic each,
    // L2 write-back and invalidate around it) takes about 16-25 us while back-to-back launches on
    // one stream are about 2.5 us apart, so chaining is off unless asked for.
    std::vector<ChainRec> chains;
    std::vector<char> in_chain(launches.size(), 0);
    const size_t chain_args_cap = chain_budget / 2 / sizeof(PassArgs);
    const size_t chain_phases_cap = chain_budget / 2 / sizeof(ChainPhase);
    if (c.tuning.chain_passes && n_paths) {
        size_t n_args = 0, n_ph = 0;
        // the phase that starts at launch j: its grid and the launch after it
        auto phase_at = [&](size_t j, unsigned &g, size_t &next) {
            const Launch &ln = launches[j];
            if (ln.kind != Launch::PASS) return false;
            g = ln.pair_next ? ln.grid + launches[j + 1].grid : ln.grid;
            next = ln.pair_next ? j + 2 : j + 1;
            return true;
        };
        for (size_t li = 0; li < launches.size();) {
            unsigned g = 0;
            size_t nx = li + 1;
            if (!phase_at(li, g, nx)) { ++li; continue; }
            const Launch &l0 = launches[li];
            const unsigned lim = chain_grid_limit(fp64, l0.R, l0.flip, c.device_cus);
            size_t j = li, na = 0;
            uint32_t np = 0;
            unsigned gmax = 0;
            while (j < launches.size()) {
                unsigned gj = 0;
                size_t nj = j + 1;
                if (!phase_at(j, gj, nj)) break;
                if (launches[j].R != l0.R || launches[j].flip != l0.flip || gj > lim) break;
                if (n_args + na + (nj - j) > chain_args_cap || n_ph + np + 1 > chain_phases_cap) break;
                na += nj - j;
                ++np;
                gmax = std::max(gmax, gj);
                j = nj;
            }
            if (np < 2) { li = nx; continue; }
            ChainRec ch;
            ch.begin = li;
            ch.end = j;
            ch.n_phases = np;
            ch.grid = gmax;
            ch.R = l0.R;
            ch.flip = l0.flip;
            ch.zskip = chain_zskip(fp64, l0.R, l0.flip);
            ch.args_first = n_args;
            ch.phases_first = n_ph;
            n_args += na;
            n_ph += np;
            for (size_t t = li; t < j; ++t) in_chain[t] = 1;
            chains.push_back(ch);
            li = j;
        }
    }
    // Row masks.  The path sum reads, per bitstring x and slot, the rows (x_h & ~vary) | m of
    // block h for every m inside vary (the qubits its fold varies: S, S' or the iSWAP qubits; none
    // for a plain gather).  The last pass of block h at that level computes a tile only if it
    // holds such a row; the tile of a row is the row with the qubits inside a tile (registers,
    // lane qubits) cleared.  Used when the tiles to compute are expected to be under 80% of the
    // state (1 - exp(-bitstrings x rows / tile positions)) and all those passes tile alike.
    bool mask_on[2] = {false, false};
    uint32_t mask_keep[2] = {0, 0}, mask_spread[2] = {0, 0};
    double mask_est[2] = {1.0, 1.0}, mask_positions[2] = {0.0, 0.0};
    if (n_paths && n_bits) {
        for (int h = 0; h < 2; ++h) {
            if (!PL.rowmask_words[h]) continue;
            uint32_t inside = 0;
            bool ok = true, any = false;
            for (const Launch &ln : launches) {
                if (!ln.row_last || ln.half != h) continue;
                const PassArgs &a = ln.pa;
                const int p = a.p_dst;
                uint32_t in = 0;
                for (int kk = 0; kk < ln.R; ++kk) {
                    if (a.reg_pos[kk] < p) ok = false;
                    else in |= 1u << (a.reg_pos[kk] - p);
                }
                const int lane_bits = a.lane_qpos4 > 0 ? 4 : a.lane_qpos > 0 ? 5 : 6;
                if (lane_bits > p) in |= (1u << (lane_bits - p)) - 1u;
                if (a.lane_qpos > 0) in |= 1u << (a.lane_qpos - p);
                if (a.lane_qpos4 > 0) in |= 1u << (a.lane_qpos4 - p);
                for (int kk = 0; kk < a.n_low; ++kk) if (a.low_pos[kk] >= p) ok = false;
                if (any && in != inside) ok = false;
                inside = in;
                any = true;
            }
            if (!any || !ok) continue;
            const uint32_t qmask = qh[h] >= 32 ? ~0u : (1u << qh[h]) - 1u;
            const uint32_t vary = !fold ? 0u : gfold ? fh[h]->g_smask : fh[h]->iswap ? fh[h]->qmask : fh[h]->smask;
            const uint32_t spread = vary & ~inside & qmask;
            if (__builtin_popcount(spread) > 6) continue;
            const double positions = std::ldexp(1.0, qh[h] - __builtin_popcount(inside & qmask));
            const double est = 1.0 - std::exp(-(double)n_bits * std::ldexp(1.0, __builtin_popcount(spread)) / positions);
            if (est > 0.8) continue;
            mask_on[h] = true;
            mask_keep[h] = qmask & ~(vary | inside);
            mask_spread[h] = spread;
            mask_est[h] = est;
            mask_positions[h] = positions;
        }
    }
    // algorithmic bytes of the masked passes at full size (scaled by the computed fraction later)
    uint64_t masked_bytes[2] = {0, 0};
    for (const Launch &ln : launches)
        if (ln.kind == Launch::PASS && ln.row_last && mask_on[ln.half]) masked_bytes[ln.half] += ln.bytes;

    if (dry_run) {
        const uint64_t rounds = n_paths ? (plain ? n_paths : 1) : 0;
        c.stats.n_sweep_launches += rounds * chains.size();
        for (size_t li = 0; li < launches.size(); ++li) {
            const Launch &ln = launches[li];
            if (ln.kind != Launch::GATHER && ln.kind != Launch::FOLD) {
                if (in_chain[li]) c.stats.n_chained_passes += rounds;
                else if (!(li > 0 && launches[li - 1].pair_next)) c.stats.n_sweep_launches += rounds;   // a pair is one launch
                c.stats.sweep_bytes += rounds * ln.bytes;
                (ln.half ? c.stats.n_passes_b : c.stats.n_passes_a)++;
            }
        }
        // planning only: every bitstring its own block-A group unless there are fewer rows
        const int kb = fold ? qh[0] - (gfold ? fh[0]->g_ns : fh[0]->iswap ? __builtin_popcount(fh[0]->qmask) : fh[0]->n_s)
                            : qh[0];
        account_gather(launches, rounds, std::min<uint64_t>(n_bits, kb >= 32 ? n_bits : (uint64_t(1) << kb)));
        c.stats.n_batches = n_leaf_batches * rounds;
        for (int h = 0; h < 2; ++h)
            c.stats.sweep_bytes -= (uint64_t)((double)(rounds * masked_bytes[h]) * (1.0 - mask_est[h]));
        return SF_OK;
    }
    if (n_paths && tables_bytes > PL.rowmask_off) { err = "internal: slot tables exceed their reservation"; return SF_ERR_UNSUPPORTED; }

    // Compiled passes (tuning jit): every pass launch outside a chain whose program (both
    // programs of a pair) the compiled form covers gets the kernel compiled for it; a repeated
    // request keeps them with its plan, other requests with the same programs find them in the
    // process-wide cache.  no_compile (the entry point without allocations: loading a kernel
    // allocates device memory for its code): only kernels already in the cache, the other passes
    // interpreted.
    if (c.tuning.jit && n_paths) {
        std::vector<std::string> srcs;
        std::vector<size_t> at;
        for (size_t li = 0; li < launches.size(); ++li) {
            Launch &ln = launches[li];
            if (ln.kind != Launch::PASS || in_chain[li] || (li > 0 && launches[li - 1].pair_next)) continue;
            if (ln.jit_fn || ln.jit_prog.empty()) continue;
            const Launch *l2 = ln.pair_next ? &launches[li + 1] : nullptr;
            if (l2 && l2->jit_prog.empty()) continue;
            auto zs = [&](const Launch &x) { return x.zskip && !fp64 && (x.R == 4 || x.R == 5); };
            srcs.push_back(jit_kernel(fp64, ln.R, ln.jit_prog, zs(ln), l2 ? l2->R : 0, l2 ? l2->jit_prog : std::string(),
                                      l2 ? zs(*l2) : false));
            at.push_back(li);
        }
        std::vector<hipFunction_t> fns;
        double ms = 0;
        if (int rc = jit_kernels(srcs, fns, &ms, err, !no_compile)) return rc;
        for (size_t i = 0; i < at.size(); ++i) launches[at[i]].jit_fn = fns[i];
        c.stats.jit_compile_ms += ms;
    }
    if (cacheable && !hit) {
        cache.valid = false;
        cache.plan = fresh;
        cache.n_paths = n_paths;
        cache.path_begin = path_begin;
        cache.n_bits = n_bits;
        cache.flags = layout_flags;
        cache.has_ids = path_ids != nullptr;
        if (path_ids) cache.ids.assign(path_ids, path_ids + n_paths);
        else cache.ids.clear();
        cache.ws = workspace;
        cache.ws_bytes = workspace_bytes;
        cache.tuning = c.tuning;
        cache.device_cus = c.device_cus;
        cache.valid = true;
    }

    // ---------------------------------------------------------------- workspace
    const size_t off_tpath = fixed;
    const size_t off_tparent = off_tpath + align_up(tpath.size() * 8);
    const size_t off_tmask = off_tparent + align_up(tparent.size() * 4);
    const size_t off_buffers = fixed + table_bound;
    size_t buffers_bytes = 0;
    for (int l = 0; l <= L; ++l)
        if (n_paths && lb[l].alias < 0 && !lb[l].none)
            buffers_bytes = std::max(buffers_bytes, lb[l].off[1] + align_up(lb[l].cap * (size_t(1) << qh[1]) * elem));
    const size_t ws_bytes = off_buffers + buffers_bytes;
    char *ws = (char *)workspace;
    if (ws) {
        if (ws_bytes > workspace_bytes) { err = "workspace too small"; return SF_ERR_OOM; }
    } else {
        if (c.dev_ws_bytes < ws_bytes) {
            if (c.dev_ws) { (void)hipFree(c.dev_ws); c.dev_ws = nullptr; c.dev_ws_bytes = 0; }
            if ((he = hipMalloc(&c.dev_ws, ws_bytes)) != hipSuccess) { err = std::string("hipMalloc: ") + hipGetErrorString(he); return SF_ERR_OOM; }
            c.dev_ws_bytes = ws_bytes;
        }
        ws = (char *)c.dev_ws;
    }

    // ---------------------------------------------------------------- enqueue
    c.stats.ms_plan = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (!pre_done) {
        const int rc = enqueue_pre(ws);
        if (rc) return rc;
    }
    double *d_acc = out_dev ? amps : (double *)(ws + off_acc);
    int *d_flag = (int *)(ws + off_flag);
    uint32_t *d_xa = (uint32_t *)(ws + off_xa), *d_xb = (uint32_t *)(ws + off_xb);
    uint32_t *d_order = (uint32_t *)(ws + off_order);
    if (!blob.empty())
        if ((he = hipMemcpyAsync(ws + off_blob, blob.data(), blob.size(), hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy plan", he);
    if (!tpath.empty()) {
        if ((he = hipMemcpyAsync(ws + off_tpath, tpath.data(), tpath.size() * 8, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy tables", he);
        if ((he = hipMemcpyAsync(ws + off_tparent, tparent.data(), tparent.size() * 4, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy tables", he);
    }
    if (!tmaskv.empty())
        if ((he = hipMemcpyAsync(ws + off_tmask, tmaskv.data(), tmaskv.size() * 4, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy masks", he);
    if (flags & SF_ACCUMULATE) {
        if (!out_dev && n_bits)
            if ((he = hipMemcpyAsync(d_acc, amps, n_bits * 16, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy amps", he);
    } else if ((he = launch_fill_zero(d_acc, 2 * (uint64_t)n_bits, stream)) != hipSuccess) {
        return dev_err("fill", he);
    }
    // row masks: cleared, marked from the bitstrings' block bits, their set bits counted
    uint32_t *d_rowmask[2] = {nullptr, nullptr};
    {
        size_t o = fixed + PL.rowmask_off;
        for (int h = 0; h < 2; ++h) {
            if (mask_on[h]) {
                d_rowmask[h] = (uint32_t *)(ws + o);
                if ((he = launch_fill_zero_i32((int *)d_rowmask[h], PL.rowmask_words[h], stream)) != hipSuccess ||
                    (he = launch_mark_rows(h ? d_xb : d_xa, n_bits, mask_keep[h], mask_spread[h], d_rowmask[h],
                                           stream)) != hipSuccess ||
                    (he = launch_count_bits(d_rowmask[h], PL.rowmask_words[h],
                                            (unsigned long long *)(d_flag + 6 + 2 * h), stream)) != hipSuccess)
                    return dev_err("row mask", he);
            }
            o += align_up(PL.rowmask_words[h] * 4);
        }
    }

    char *buf = ws + off_buffers;
    auto pass_args = [&](const Launch &ln) {
        PassArgs a = ln.pa;
        a.dst = buf + ln.dst_off;
        a.src = buf + ln.src_off;
        a.slot_path = (const uint64_t *)(ws + off_tpath) + ln.table_off;
        a.slot_parent = (const uint32_t *)(ws + off_tparent) + ln.table_off;
        a.slot_parent_base = 0;
        a.prog = (const uint32_t *)(ws + off_blob + ln.plan_off);
        a.row_mask = ln.row_last ? d_rowmask[ln.half] : nullptr;
        a.prog_words = ln.prog_words;
        a.groups_word = ln.groups_word;
        a.terms_word = ln.terms_word;
        return a;
    };
    // the chains' pass arguments and phases (the same for every round: the plain form rewrites
    // the slot tables in place)
    const PassArgs *d_chain_args = (const PassArgs *)(ws + off_chain);
    const ChainPhase *d_chain_phases = (const ChainPhase *)(ws + off_chain + chain_budget / 2);
    uint64_t *d_bar = (uint64_t *)(d_flag + 4);
    std::vector<PassArgs> chain_args;
    std::vector<ChainPhase> chain_phases;
    for (const ChainRec &ch : chains) {
        if (chain_phases.size() != ch.phases_first || chain_args.size() != ch.args_first) {
            err = "internal: chained launch tables out of order";
            return SF_ERR_UNSUPPORTED;
        }
        for (size_t j = ch.begin; j < ch.end;) {
            const Launch &ln = launches[j];
            ChainPhase ph{};
            ph.first = (uint32_t)chain_args.size();     // index into the whole array
            chain_args.push_back(pass_args(ln));
            if (ln.pair_next) {
                const Launch &l2 = launches[j + 1];
                chain_args.push_back(pass_args(l2));
                const uint64_t g0 = ln.grid, gs = (uint64_t)ln.grid + l2.grid;
                const uint64_t split = (ch.grid * g0 + gs / 2) / gs;
                ph.n = 2;
                ph.split = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(split, 1), ch.grid - 1);
                j += 2;
            } else {
                ph.n = 1;
                j += 1;
            }
            chain_phases.push_back(ph);
        }
    }
    if (chain_args.size() > chain_args_cap || chain_phases.size() > chain_phases_cap) {
        err = "internal: chained launches exceed their reservation";
        return SF_ERR_UNSUPPORTED;
    }
    if (!chain_args.empty()) {
        if ((he = hipMemcpyAsync(ws + off_chain, chain_args.data(), chain_args.size() * sizeof(PassArgs),
                                 hipMemcpyHostToDevice, stream)) != hipSuccess)
            return dev_err("copy chains", he);
        if ((he = hipMemcpyAsync(ws + off_chain + chain_budget / 2, chain_phases.data(),
                                 chain_phases.size() * sizeof(ChainPhase), hipMemcpyHostToDevice, stream)) != hipSuccess)
            return dev_err("copy chains", he);
    }
    uint64_t bar_base = 0;
    const uint64_t rounds = n_paths ? (plain ? n_paths : 1) : 0;
    for (uint64_t r = 0; r < rounds; ++r) {
        if (plain && r > 0) {
            // same launch sequence with the slot tables of the next path
            const uint64_t pid = path_ids ? path_ids[r] : path_begin + r;
            for (const BatchRec &b : batches) {
                const int drop = k - c.levels[b.level].bits_after;
                const uint64_t v = drop >= 64 ? 0 : ((pid >> drop) << drop);
                for (uint64_t i = 0; i < b.slots; ++i) tpath[b.table_off + i] = v;
            }
            if (plain_mask_idx != SIZE_MAX) {
                const uint64_t m = uint64_t(1) << (pid & ((uint64_t(1) << fh[0]->nb) - 1));
                tmaskv[plain_mask_idx] = (uint32_t)m;
                if (fh[0]->iswap) tmaskv[plain_mask_idx + 1] = (uint32_t)(m >> 32);
            }
            // the previous path's launches must be done with the old tables
            if ((he = hipStreamSynchronize(stream)) != hipSuccess) return dev_err("sync", he);
            if ((he = hipMemcpy(ws + off_tpath, tpath.data(), tpath.size() * 8, hipMemcpyHostToDevice)) != hipSuccess) return dev_err("copy tables", he);
            if (!tmaskv.empty())
                if ((he = hipMemcpy(ws + off_tmask, tmaskv.data(), tmaskv.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) return dev_err("copy masks", he);
        }
        int cur_cat = -1, cur_id = -1;     // open event pair: a run of launches of one category
        auto timed = [&](int cat) {
            if (!timing || cat == cur_cat) return;
            ev_end(cur_id);
            cur_id = ev_begin(cat);
            cur_cat = cat;
        };
        size_t ci = 0;    // next chain
        for (size_t li = 0; li < launches.size(); ++li) {
            const Launch &ln = launches[li];
            if (ci < chains.size() && li == chains[ci].begin) {
                const ChainRec &ch = chains[ci++];
                timed(0);
                // phases index the call's whole argument array; each chain reads its own phases
                if ((he = launch_pass_chain(fp64, ch.R, ch.flip, ch.zskip, d_chain_args, d_chain_phases + ch.phases_first, ch.n_phases, d_bar, bar_base, d_flag + 2,
                                            ch.grid, stream)) != hipSuccess)
                    return dev_err("chained passes", he);
                bar_base += (uint64_t)(ch.n_phases - 1) * ch.grid;
                c.stats.n_sweep_launches++;
                c.stats.n_chained_passes += ch.end - ch.begin;
                for (size_t t = ch.begin; t < ch.end; ++t) c.stats.sweep_bytes += launches[t].bytes;
                li = ch.end - 1;
                continue;
            }
            if (ln.kind == Launch::PASS && ln.pair_next) {
                const Launch &l2 = launches[li + 1];
                timed(0);
                if (ln.jit_fn) {
                    PassArgs a0 = pass_args(ln), a1 = pass_args(l2);
                    uint32_t g0 = ln.grid;
                    void *kp[] = {&a0, &a1, &g0};
                    if ((he = hipModuleLaunchKernel(ln.jit_fn, ln.grid + l2.grid, 1, 1, 256, 1, 1, 0, stream, kp,
                                                    nullptr)) != hipSuccess)
                        return dev_err("compiled pass", he);
                    c.stats.n_jit_passes += 2;
                } else if ((he = launch_pass_pair(fp64, ln.R, ln.flip, ln.zskip || l2.zskip, pass_args(ln), ln.grid,
                                                  pass_args(l2), l2.grid, stream)) != hipSuccess) {
                    return dev_err("pass", he);
                }
                c.stats.n_sweep_launches++;
                c.stats.sweep_bytes += ln.bytes + l2.bytes;
                ++li;
                continue;
            }
            if (ln.kind == Launch::DENSE) {
                DenseArgs d = ln.da;
                d.dst = buf + ln.dst_off;
                d.src = buf + ln.src_off;
                d.mat = (const float *)(ws + off_blob + ln.plan_off);
                timed(0);
                if ((he = launch_dense(d, ln.grid, stream)) != hipSuccess) return dev_err("dense", he);
                c.stats.n_sweep_launches++;
                c.stats.sweep_bytes += ln.bytes;
            } else if (ln.kind == Launch::PASS) {
                timed(0);
                if (ln.jit_fn) {
                    PassArgs a0 = pass_args(ln);
                    void *kp[] = {&a0};
                    if ((he = hipModuleLaunchKernel(ln.jit_fn, ln.grid, 1, 1, 256, 1, 1, 0, stream, kp, nullptr)) != hipSuccess)
                        return dev_err("compiled pass", he);
                    c.stats.n_jit_passes++;
                } else if ((he = launch_pass(fp64, ln.R, ln.flip, ln.zskip, pass_args(ln), ln.grid, stream)) != hipSuccess) {
                    return dev_err("pass", he);
                }
                c.stats.n_sweep_launches++;
                c.stats.sweep_bytes += ln.bytes;
            } else if (ln.kind == Launch::FOLD && fh[0]->iswap) {
                FoldIswapArgs f = ln.fia;
                f.h[0].par = buf + ln.dst_off;
                f.h[1].par = buf + ln.src_off;
                for (int h = 0; h < 2; ++h) f.h[h].tab = (const double *)(ws + off_blob + fold_tab_off[h]);
                f.xa = d_xa;
                f.xb = d_xb;
                f.order = d_order;
                f.acc = d_acc;
                f.child_mask = (const uint64_t *)((const uint32_t *)(ws + off_tmask) + ln.mask_off);
                timed(1);
                if ((he = launch_fold_iswap(fp64, fh[0]->ng, f, stream)) != hipSuccess) return dev_err("fold", he);
            } else if (ln.kind == Launch::FOLD && gfold) {
                GFoldArgs f = ln.gfa;
                f.h[0].par = buf + ln.dst_off;
                f.h[1].par = buf + ln.src_off;
                if (ln.defer) {
                    const uint32_t *tm = (const uint32_t *)(ws + off_tmask);
                    f.h[0].par_slot = tm + ln.dpar_off;
                    f.h[0].dsub = tm + ln.dsub_off;
                    f.h[0].dfac = tm + ln.dfac_off;
                }
                for (int h = 0; h < 2; ++h) {
                    f.h[h].tab = ws + off_blob + fold_tab_off[h];
                    f.h[h].off = (const uint32_t *)(ws + off_blob + PL.fold_off_off[h]);
                }
                f.xa = d_xa;
                f.xb = d_xb;
                f.order = d_order;
                f.acc = d_acc;
                f.child_mask = (const uint32_t *)(ws + off_tmask) + ln.mask_off;
                timed(1);
                if ((he = launch_gfold(fp64, fh[0]->nb, f, stream)) != hipSuccess) return dev_err("fold", he);
            } else if (ln.kind == Launch::FOLD) {
                FoldArgs f = ln.fa;
                f.h[0].par = buf + ln.dst_off;
                f.h[1].par = buf + ln.src_off;
                for (int h = 0; h < 2; ++h) f.h[h].tab = (const double *)(ws + off_blob + fold_tab_off[h]);
                f.xa = d_xa;
                f.xb = d_xb;
                f.order = d_order;
                f.acc = d_acc;
                f.child_mask = (const uint32_t *)(ws + off_tmask) + ln.mask_off;
                timed(1);
                if ((he = launch_fold(fp64, fh[0]->nb, f, stream)) != hipSuccess) return dev_err("fold", he);
            } else {
                GatherArgs g = ln.ga;
                g.a = buf + ln.dst_off;
                g.b = buf + ln.src_off;
                g.xa = d_xa;
                g.xb = d_xb;
                g.order = d_order;
                g.acc = d_acc;
                timed(1);
                if ((he = launch_gather(fp64, g, stream)) != hipSuccess) return dev_err("gather", he);
            }
        }
        ev_end(cur_id);
    }
    if (!out_dev && n_bits)
        if ((he = hipMemcpyAsync(amps, d_acc, n_bits * 16, hipMemcpyDeviceToHost, stream)) != hipSuccess) return dev_err("copy amps", he);
    int flag[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if ((he = hipMemcpyAsync(flag, d_flag, sizeof(flag), hipMemcpyDeviceToHost, stream)) != hipSuccess) return dev_err("copy flag", he);
    if ((he = hipStreamSynchronize(stream)) != hipSuccess) return dev_err("synchronize", he);
    if (flag[0]) { err = "bitstring has bits outside the grid"; return SF_ERR_INVALID; }
    if (flag[2]) {
        err = "a chained launch's grid barrier did not complete (its workgroups were not all resident); "
              "chain_passes = 0 runs one launch per pass";
        return SF_ERR_DEVICE;
    }
    account_gather(launches, rounds, (uint64_t)flag[1]);
    // the masked passes moved the bytes of the tiles they computed
    for (int h = 0; h < 2; ++h) {
        if (!mask_on[h]) continue;
        uint64_t set = 0;
        std::memcpy(&set, flag + 6 + 2 * h, 8);
        const double frac = std::min(1.0, (double)set / mask_positions[h]);
        c.stats.sweep_bytes -= (uint64_t)((double)(rounds * masked_bytes[h]) * (1.0 - frac));
        c.stats.row_mask_frac[h] = frac;
    }

    if (timing) {
        for (size_t i = 0; i < ev_cat.size(); ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, (hipEvent_t)c.events[2 * i], (hipEvent_t)c.events[2 * i + 1]);
            if (ev_cat[i] == 0) c.stats.ms_sweep += ms;
            else if (ev_cat[i] == 1) c.stats.ms_gather += ms;
            else c.stats.ms_other += ms;
        }
    }
    c.stats.n_batches = n_leaf_batches * (plain ? n_paths : 1);
    for (const Launch &ln : launches)
        if (ln.kind != Launch::GATHER && ln.kind != Launch::FOLD) (ln.half ? c.stats.n_passes_b : c.stats.n_passes_a)++;
    c.stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return SF_OK;
}

}  // namespace sf
