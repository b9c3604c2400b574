// Executor: prefix tree of the requested paths, batches that fit the
// workspace, and the launch sequence (passes per tree level, fan-out
// copies with the branch operators, gather + FP64 path sum at the leaves).
//
// The paper keeps one checkpoint per process after the x_p-bit prefix and
// replays 2^x_b branches from it (Section 2); its logs show a second
// checkpoint level ("p + r + b").  Here every clock cycle that holds
// crossing CZs is a tree level: the nodes of a level are the distinct
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
    std::vector<uint64_t> leaf(n);
    if (ids) {
        std::copy(ids, ids + n, leaf.begin());
        std::sort(leaf.begin(), leaf.end());
        for (uint64_t i = 1; i < n; ++i)
            if (leaf[i] == leaf[i - 1]) { err = "path ids must be distinct"; return SF_ERR_INVALID; }
    } else {
        for (uint64_t i = 0; i < n; ++i) leaf[i] = begin + i;
    }
    if (n && (k < 64) && (leaf.back() >> k) != 0) { err = "path id >= 2^k"; return SF_ERR_INVALID; }
    t.node.assign(L + 1, {});
    t.parent.assign(L + 1, {});
    t.first_child.assign(L + 1, {});
    for (int l = 0; l <= L; ++l) {
        const int drop = k - c.levels[l].bits_after;   // bits not yet decided at this level
        std::vector<uint64_t> &nd = t.node[l];
        for (uint64_t i = 0; i < n; ++i) {
            const uint64_t v = drop >= 64 ? 0 : ((leaf[i] >> drop) << drop);
            if (nd.empty() || nd.back() != v) nd.push_back(v);
        }
        if (l > 0) {
            const int pdrop = k - c.levels[l - 1].bits_after;
            std::vector<uint32_t> &par = t.parent[l];
            par.resize(nd.size());
            const std::vector<uint64_t> &pn = t.node[l - 1];
            size_t pi = 0;
            for (size_t i = 0; i < nd.size(); ++i) {
                const uint64_t pv = pdrop >= 64 ? 0 : ((nd[i] >> pdrop) << pdrop);
                while (pn[pi] != pv) ++pi;
                par[i] = (uint32_t)pi;
            }
            std::vector<uint64_t> &fc = t.first_child[l - 1];
            fc.assign(pn.size() + 1, 0);
            for (size_t i = 0; i < nd.size(); ++i) fc[par[i] + 1]++;
            for (size_t i = 0; i < pn.size(); ++i) fc[i + 1] += fc[i];
        }
    }
    return SF_OK;
}

struct LevelBuf {
    int alias = -1;       // level whose buffer this level reuses in place (chain levels)
    uint64_t cap = 1;     // slots
    size_t off[2] = {0, 0};
};

struct Launch {
    enum Kind { PASS, GATHER } kind;
    int half = 0;
    int R = 0;
    PassArgs pa{};
    GatherArgs ga{};
    size_t plan_off = 0;      // device offset of the pass program inside the plan blob
    uint32_t prog_words = 0, groups_word = 0, terms_word = 0;
    int level = 0;
    size_t dst_off = 0, src_off = 0;
    size_t slot_off = 0;      // element offset into the level's node / parent tables
    uint32_t parent_base = 0;
    unsigned grid = 1;
    uint64_t bytes = 0;
};

struct BlobEntry { size_t off; uint32_t words, groups_word, terms_word; };

}  // namespace

int estimate_workspace(const Circuit &c, uint64_t n_paths, size_t n_bits, uint32_t flags, size_t *bytes)
{
    const size_t elem = (flags & SF_FP64_SWEEPS) ? 16 : 8;
    const size_t sigma = (size_t(1) << c.half[0].q) * elem + (size_t(1) << c.half[1].q) * elem;
    const int L = (int)c.levels.size() - 1;
    // upper bound: every level resident with min(2^bits, n_paths) nodes
    size_t total = 0;
    for (int l = 0; l <= L; ++l) {
        const int b = c.levels[l].bits_after;
        uint64_t nodes = b >= 63 ? n_paths : std::min<uint64_t>(uint64_t(1) << b, n_paths);
        total += next_pow2(std::max<uint64_t>(nodes, 1)) * sigma;
        total += align_up(nodes * 12 + 64 * 12) ;
    }
    total += align_up(n_bits * 8) * 2 + align_up(n_bits * 16) + (size_t(1) << 22);
    *bytes = total;
    return SF_OK;
}

int execute(Circuit &c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
            const uint64_t *bits, size_t n_bits, double *amps, uint32_t flags, void *stream_v,
            void *workspace, size_t workspace_bytes, std::string &err)
{
    const auto t_start = std::chrono::steady_clock::now();
    hipStream_t stream = (hipStream_t)stream_v;
    const bool fp64 = (flags & SF_FP64_SWEEPS) != 0;
    const bool plain = (flags & SF_PLAIN) != 0;
    const bool timing = (flags & SF_TIMING) != 0;
    const size_t elem = fp64 ? 16 : 8;
    const int L = (int)c.levels.size() - 1;
    const int qh[2] = {c.half[0].q, c.half[1].q};
    int R = c.tuning.reg_qubits ? (int)c.tuning.reg_qubits : kMaxRegBits;
    R = std::max(1, std::min(R, fp64 ? kMaxRegBitsF64 : kMaxRegBits));
    c.stats = sf_run_stats_t{};

    if (!path_ids && n_paths && c.k < 64 && ((path_begin + n_paths - 1) >> c.k) != 0) {
        err = "path range exceeds 2^k";
        return SF_ERR_INVALID;
    }
    const uint64_t all = c.n == 64 ? ~uint64_t(0) : ((uint64_t(1) << c.n) - 1);
    if (!(flags & SF_BITS_ON_DEVICE)) {
        for (size_t j = 0; j < n_bits; ++j)
            if (bits[j] & ~all) { err = "bitstring has bits outside the grid"; return SF_ERR_INVALID; }
    }

    hipError_t he;
    int dev = 0;
    if ((he = hipGetDevice(&dev)) != hipSuccess) { err = std::string("hipGetDevice: ") + hipGetErrorString(he); return SF_ERR_DEVICE; }
    if (!c.device_cus) {
        if ((he = hipDeviceGetAttribute(&c.device_cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) {
            err = std::string("hipDeviceGetAttribute: ") + hipGetErrorString(he);
            return SF_ERR_DEVICE;
        }
    }

    // ---------------------------------------------------------------- tree
    // In plain form every path is its own tree (one node per level, no sharing).
    const uint64_t n_trees = plain ? n_paths : (n_paths ? 1 : 0);

    // min slots so that every block state has at least 6 extended bits (one wave of lanes)
    const int qmin = std::min(qh[0], qh[1]);
    const uint64_t min_slots = qmin >= 6 ? 1 : (uint64_t(1) << (6 - qmin));

    // ---------------------------------------------------------------- fixed workspace parts
    const size_t sigma = (size_t(1) << qh[0]) * elem + (size_t(1) << qh[1]) * elem;
    const bool bits_dev = (flags & SF_BITS_ON_DEVICE) != 0;
    const bool out_dev = (flags & SF_OUT_ON_DEVICE) != 0;
    size_t fixed = 0;
    const size_t off_xa = fixed; fixed += align_up(n_bits * 4);
    const size_t off_xb = fixed; fixed += align_up(n_bits * 4);
    const size_t off_bits = fixed; if (!bits_dev) fixed += align_up(n_bits * 8);
    const size_t off_acc = fixed; if (!out_dev) fixed += align_up(n_bits * 16);
    const size_t off_flag = fixed; fixed += kAlign;

    // Builds the launch list for one tree; returns the workspace bytes it needs.
    struct RunPlan {
        Tree tree;
        std::vector<LevelBuf> lb;
        std::vector<size_t> table_off;        // per level: byte offset of node table, parent table
        std::vector<size_t> parent_table_off;
        size_t tables_bytes = 0, buffers_bytes = 0;
    };

    auto plan_levels = [&](RunPlan &rp, size_t budget) -> int {
        const Tree &t = rp.tree;
        rp.lb.assign(L + 1, LevelBuf{});
        // chain levels (each parent has exactly one child) reuse the parent's buffer in place
        for (int l = 1; l <= L; ++l)
            if (t.node[l].size() == t.node[l - 1].size()) rp.lb[l].alias = rp.lb[l - 1].alias >= 0 ? rp.lb[l - 1].alias : l - 1;
        uint64_t maxs = c.tuning.max_slots ? c.tuning.max_slots : (uint64_t(1) << 20);
        uint64_t leafmax = c.tuning.leaf_batch ? c.tuning.leaf_batch : maxs;
        for (int l = 0; l <= L; ++l) {
            uint64_t want = next_pow2(std::max<uint64_t>(t.node[l].size(), 1));
            want = std::min(want, l == L ? leafmax : maxs);
            rp.lb[l].cap = std::max(want, min_slots);
        }
        // shrink the largest owned buffers until everything fits
        for (;;) {
            for (int l = 1; l <= L; ++l) if (rp.lb[l].alias >= 0) rp.lb[l].cap = rp.lb[rp.lb[l].alias].cap;
            size_t need = 0;
            for (int l = 0; l <= L; ++l) if (rp.lb[l].alias < 0) need += rp.lb[l].cap * sigma;
            if (need + rp.tables_bytes <= budget) { rp.buffers_bytes = need; break; }
            int big = -1;
            for (int l = 0; l <= L; ++l)
                if (rp.lb[l].alias < 0 && rp.lb[l].cap > min_slots && (big < 0 || rp.lb[l].cap >= rp.lb[big].cap)) big = l;
            if (big < 0) return SF_ERR_OOM;
            rp.lb[big].cap >>= 1;
        }
        return SF_OK;
    };

    // ---------------------------------------------------------------- workspace
    std::vector<RunPlan> plans(n_trees ? 1 : 0);
    int rc;
    size_t ws_bytes = workspace ? workspace_bytes : 0;
    if (n_trees) {
        RunPlan &rp = plans[0];
        if (plain) {
            const uint64_t first = path_ids ? path_ids[0] : path_begin;
            if ((rc = build_tree(c, &first, 0, 1, rp.tree, err))) return rc;
            if (path_ids) {
                for (uint64_t i = 0; i < n_paths; ++i)
                    if (c.k < 64 && (path_ids[i] >> c.k)) { err = "path id >= 2^k"; return SF_ERR_INVALID; }
            }
        } else {
            if ((rc = build_tree(c, path_ids, path_begin, n_paths, rp.tree, err))) return rc;
        }
        rp.tables_bytes = 0;
        rp.table_off.assign(L + 1, 0);
        rp.parent_table_off.assign(L + 1, 0);
    }
    // tables are padded by the largest batch so padded slots read valid entries
    auto tables_size = [&](RunPlan &rp) {
        size_t tb = 0;
        for (int l = 0; l <= L; ++l) {
            const size_t nn = rp.tree.node[l].size() + rp.lb[l].cap;
            rp.table_off[l] = tb; tb += align_up(nn * 8);
            rp.parent_table_off[l] = tb; tb += align_up(nn * 4);
        }
        return tb;
    };

    size_t plan_blob_budget = size_t(1) << 22;   // grown below if needed
    if (n_trees) {
        RunPlan &rp = plans[0];
        // first guess of the table size with caps of the node counts
        rp.lb.assign(L + 1, LevelBuf{});
        for (int l = 0; l <= L; ++l) rp.lb[l].cap = std::max<uint64_t>(next_pow2(std::max<size_t>(rp.tree.node[l].size(), 1)), min_slots);
        rp.tables_bytes = tables_size(rp);
        size_t budget;
        if (workspace) {
            if (workspace_bytes < fixed + plan_blob_budget + rp.tables_bytes) { err = "workspace too small"; return SF_ERR_OOM; }
            budget = workspace_bytes - fixed - plan_blob_budget;
        } else {
            size_t free_b = 0, total_b = 0;
            if ((he = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) { err = std::string("hipMemGetInfo: ") + hipGetErrorString(he); return SF_ERR_DEVICE; }
            const size_t avail = c.dev_ws_bytes + (size_t)(0.85 * (double)free_b);
            if (avail < fixed + plan_blob_budget) { err = "not enough device memory"; return SF_ERR_OOM; }
            budget = avail - fixed - plan_blob_budget;
        }
        if ((rc = plan_levels(rp, budget))) { err = "workspace too small for one slot per tree level"; return rc; }
        rp.tables_bytes = tables_size(rp);
        ws_bytes = fixed + plan_blob_budget + rp.tables_bytes + rp.buffers_bytes;
        if (workspace && ws_bytes > workspace_bytes) {
            // tables grew with the final caps; shrink once more
            if ((rc = plan_levels(rp, workspace_bytes - fixed - plan_blob_budget))) { err = "workspace too small"; return rc; }
            rp.tables_bytes = tables_size(rp);
            ws_bytes = fixed + plan_blob_budget + rp.tables_bytes + rp.buffers_bytes;
            if (ws_bytes > workspace_bytes) { err = "workspace too small"; return SF_ERR_OOM; }
        }
    } else {
        ws_bytes = fixed + kAlign;
    }

    char *ws = (char *)workspace;
    if (!ws) {
        if (c.dev_ws_bytes < ws_bytes) {
            if (c.dev_ws) { (void)hipFree(c.dev_ws); c.dev_ws = nullptr; c.dev_ws_bytes = 0; }
            if ((he = hipMalloc(&c.dev_ws, ws_bytes)) != hipSuccess) {
                err = std::string("hipMalloc: ") + hipGetErrorString(he);
                return SF_ERR_OOM;
            }
            c.dev_ws_bytes = ws_bytes;
        }
        ws = (char *)c.dev_ws;
    }
    const size_t off_blob = fixed;
    const size_t off_tables = off_blob + plan_blob_budget;

    // ---------------------------------------------------------------- launch list
    std::vector<Launch> launches;
    bool plan_error = false;
    std::vector<char> blob;                    // host image of the plan blob
    std::map<const SegmentPlan *, std::vector<BlobEntry>> blob_index;
    std::complex<double> leaf_scale[2];
    for (int h = 0; h < 2; ++h) {
        std::complex<double> s = c.half[h].init_scale;
        for (int l = 0; l <= L; ++l) s *= c.half[h].seg_scale[l];
        leaf_scale[h] = s;
    }
    const std::complex<double> gscale = leaf_scale[0] * leaf_scale[1];

    auto blob_put = [&](const void *p, size_t nbytes) {
        const size_t o = align_up(blob.size());
        blob.resize(o + nbytes);
        if (nbytes) std::memcpy(blob.data() + o, p, nbytes);
        return o;
    };
    auto blob_entries = [&](const SegmentPlan &sp) -> const std::vector<BlobEntry> & {
        auto it = blob_index.find(&sp);
        if (it != blob_index.end()) return it->second;
        std::vector<BlobEntry> v;
        for (const PassPlan &pp : sp.passes) {
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
            if (e.words > (uint32_t)kMaxProgWords) { plan_error = true; }
            e.off = blob_put(img.data(), img.size());
            v.push_back(e);
        }
        return blob_index.emplace(&sp, std::move(v)).first->second;
    };

    const unsigned max_grid = (unsigned)std::max(1, c.device_cus) * (c.tuning.waves_per_cu ? c.tuning.waves_per_cu / 4 : 8);
    uint64_t n_batches = 0;

    // enqueue the passes of segment `level` for one batch of nslots slots
    auto add_segment = [&](RunPlan &rp, int level, uint64_t nslots, size_t dst_base[2], int src_level,
                           size_t src_base[2], uint64_t src_slots, size_t slot_first, uint32_t parent_base,
                           bool first_from_init) {
        const int p = log2u(nslots);
        const int ps = log2u(src_slots);
        for (int h = 0; h < 2; ++h) {
            const SegmentPlan &sp = get_segment_plan(c, h, level, p, R);
            if (!sp.ok) { plan_error = true; return; }
            const std::vector<BlobEntry> &be = blob_entries(sp);
            const int n_ext = p + qh[h];
            for (size_t i = 0; i < sp.passes.size(); ++i) {
                const PassPlan &pp = sp.passes[i];
                Launch ln;
                ln.kind = Launch::PASS;
                ln.half = h;
                ln.R = pp.R;
                ln.level = level;
                PassArgs &a = ln.pa;
                std::memset(&a, 0, sizeof(a));
                a.n_tiles = uint64_t(1) << (n_ext - 6 - pp.R);
                a.n_ops = (uint32_t)pp.ops.size();
                a.p_dst = p;
                a.p_src = p;
                a.src_mode = SRC_SAME;
                a.rescale = std::ldexp(1.0, -pp.rescale_exp);
                for (int k = 0; k < 6; ++k) a.reg_pos[k] = pp.reg_pos[k];
                ln.dst_off = dst_base[h];
                ln.src_off = dst_base[h];
                if (i == 0 && first_from_init) {
                    a.src_mode = SRC_INIT;
                    uint64_t z = 0;
                    for (int t = 0; t < qh[h]; ++t)
                        if (!((c.half[h].init_h_mask >> t) & 1)) z |= uint64_t(1) << (p + t);
                    a.init_zero_mask = z;
                } else if (i == 0 && src_level >= 0) {
                    a.src_mode = SRC_FANOUT;
                    a.p_src = ps;
                    ln.src_off = src_base[h];
                }
                ln.slot_off = slot_first;
                ln.parent_base = parent_base;
                ln.plan_off = be[i].off;
                ln.prog_words = be[i].words;
                ln.groups_word = be[i].groups_word;
                ln.terms_word = be[i].terms_word;
                const uint64_t waves = a.n_tiles;
                ln.grid = (unsigned)std::min<uint64_t>((waves + 3) / 4, max_grid);
                ln.bytes = (uint64_t(1) << n_ext) * elem * (a.src_mode == SRC_INIT ? 1 : 2);
                launches.push_back(ln);
            }
        }
    };

    // depth-first over batches
    std::function<void(RunPlan &, int, uint64_t, uint64_t, uint64_t)> visit;
    visit = [&](RunPlan &rp, int l, uint64_t lo, uint64_t hi, uint64_t nslots) {
        if (plan_error) return;
        const LevelBuf &me = rp.lb[l];
        const int own = me.alias >= 0 ? me.alias : l;
        if (l == L) {
            Launch ln;
            ln.kind = Launch::GATHER;
            ln.level = l;
            GatherArgs &g = ln.ga;
            std::memset(&g, 0, sizeof(g));
            g.n_bits = n_bits;
            g.n_slots = (uint32_t)(hi - lo);
            g.p = log2u(nslots);
            g.scale_re = gscale.real();
            g.scale_im = gscale.imag();
            ln.dst_off = rp.lb[own].off[0];
            ln.src_off = rp.lb[own].off[1];
            ln.bytes = (uint64_t)n_bits * (uint64_t)(hi - lo) * 2 * elem;
            launches.push_back(ln);
            ++n_batches;
            return;
        }
        const std::vector<uint64_t> &fc = rp.tree.first_child[l];
        const uint64_t clo = fc[lo], chi = fc[hi];
        const LevelBuf &cb = rp.lb[l + 1];
        if (cb.alias >= 0) {
            // chain level: same nodes one-to-one, evolve in place
            size_t base[2] = {rp.lb[own].off[0], rp.lb[own].off[1]};
            add_segment(rp, l + 1, nslots, base, -1, base, nslots, clo, 0, false);
            visit(rp, l + 1, clo, chi, nslots);
            return;
        }
        size_t src[2] = {rp.lb[own].off[0], rp.lb[own].off[1]};
        for (uint64_t a = clo; a < chi; a += cb.cap) {
            const uint64_t b = std::min(chi, a + cb.cap);
            const uint64_t ns = std::max<uint64_t>(next_pow2(b - a), min_slots);
            size_t dst[2] = {cb.off[0], cb.off[1]};
            add_segment(rp, l + 1, ns, dst, l, src, nslots, a, (uint32_t)lo, false);
            visit(rp, l + 1, a, b, ns);
            if (plan_error) return;
        }
    };

    if (n_trees) {
        RunPlan &rp = plans[0];
        size_t o = off_tables + rp.tables_bytes;
        for (int l = 0; l <= L; ++l) {
            if (rp.lb[l].alias >= 0) continue;
            for (int h = 0; h < 2; ++h) {
                rp.lb[l].off[h] = o;
                o += align_up(rp.lb[l].cap * (size_t(1) << qh[h]) * elem);
            }
        }
        for (int l = 0; l <= L; ++l)
            if (rp.lb[l].alias >= 0) { rp.lb[l].off[0] = rp.lb[rp.lb[l].alias].off[0]; rp.lb[l].off[1] = rp.lb[rp.lb[l].alias].off[1]; }
        // root batch
        const uint64_t ns0 = std::max<uint64_t>(1, min_slots);
        size_t base0[2] = {rp.lb[0].off[0], rp.lb[0].off[1]};
        add_segment(rp, 0, ns0, base0, -1, base0, ns0, 0, 0, true);
        visit(rp, 0, 0, 1, ns0);
    }
    if (plan_error) { err = "internal: a segment could not be scheduled into passes"; return SF_ERR_UNSUPPORTED; }
    if (blob.size() > plan_blob_budget) { err = "internal: plan blob larger than its reservation"; return SF_ERR_UNSUPPORTED; }

    // ---------------------------------------------------------------- host images of the tables
    std::vector<char> tables;
    if (n_trees) {
        RunPlan &rp = plans[0];
        tables.assign(rp.tables_bytes, 0);
        for (int l = 0; l <= L; ++l) {
            const std::vector<uint64_t> &nd = rp.tree.node[l];
            uint64_t *pt = (uint64_t *)(tables.data() + rp.table_off[l]);
            uint32_t *pp = (uint32_t *)(tables.data() + rp.parent_table_off[l]);
            const size_t nn = nd.size() + rp.lb[l].cap;
            for (size_t i = 0; i < nn; ++i) {
                pt[i] = nd[std::min(i, nd.size() - 1)];
                pp[i] = l ? rp.tree.parent[l][std::min(i, nd.size() - 1)] : 0;
            }
        }
    }

    // ---------------------------------------------------------------- enqueue
    auto dev_err = [&](const char *what, hipError_t e) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return SF_ERR_DEVICE;
    };
    const uint64_t *d_bits = bits_dev ? bits : (const uint64_t *)(ws + off_bits);
    double *d_acc = out_dev ? amps : (double *)(ws + off_acc);
    int *d_flag = (int *)(ws + off_flag);
    uint32_t *d_xa = (uint32_t *)(ws + off_xa), *d_xb = (uint32_t *)(ws + off_xb);

    std::vector<hipEvent_t> ev;
    std::vector<int> ev_cat;    // 0 sweep, 1 gather, 2 other
    auto ev_pair = [&](int cat) -> hipEvent_t * {
        if (!timing) return nullptr;
        ev.emplace_back();
        ev.emplace_back();
        (void)hipEventCreate(&ev[ev.size() - 2]);
        (void)hipEventCreate(&ev[ev.size() - 1]);
        ev_cat.push_back(cat);
        return &ev[ev.size() - 2];
    };

    if (!bits_dev && n_bits)
        if ((he = hipMemcpyAsync((void *)d_bits, bits, n_bits * 8, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy bitstrings", he);
    if (!blob.empty())
        if ((he = hipMemcpyAsync(ws + off_blob, blob.data(), blob.size(), hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy plan", he);
    if (!tables.empty())
        if ((he = hipMemcpyAsync(ws + off_tables, tables.data(), tables.size(), hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy tables", he);
    {
        hipEvent_t *e = ev_pair(2);
        if (e) (void)hipEventRecord(e[0], stream);
        if ((he = launch_fill_zero_i32(d_flag, 1, stream)) != hipSuccess) return dev_err("fill", he);
        if ((he = launch_pext(d_bits, n_bits, c.mask_a, c.mask_b, all, d_xa, d_xb, d_flag, stream)) != hipSuccess) return dev_err("pext", he);
        if (flags & SF_ACCUMULATE) {
            if (!out_dev && n_bits)
                if ((he = hipMemcpyAsync(d_acc, amps, n_bits * 16, hipMemcpyHostToDevice, stream)) != hipSuccess) return dev_err("copy amps", he);
        } else {
            if ((he = launch_fill_zero(d_acc, 2 * (uint64_t)n_bits, stream)) != hipSuccess) return dev_err("fill", he);
        }
        if (e) (void)hipEventRecord(e[1], stream);
    }

    const uint64_t trees_to_run = n_trees;
    for (uint64_t tr = 0; tr < trees_to_run; ++tr) {
        RunPlan &rp = plans[0];
        if (plain && tr > 0) {
            // same launch sequence, slot tables of the next path
            const uint64_t pid = path_ids ? path_ids[tr] : path_begin + tr;
            std::vector<char> tb(rp.tables_bytes, 0);
            for (int l = 0; l <= L; ++l) {
                const int drop = c.k - c.levels[l].bits_after;
                const uint64_t v = drop >= 64 ? 0 : ((pid >> drop) << drop);
                uint64_t *pt = (uint64_t *)(tb.data() + rp.table_off[l]);
                uint32_t *pp = (uint32_t *)(tb.data() + rp.parent_table_off[l]);
                const size_t nn = 1 + rp.lb[l].cap;
                for (size_t i = 0; i < nn; ++i) { pt[i] = v; pp[i] = 0; }
            }
            // synchronous copy: the previous path's launches must have consumed the old tables
            if ((he = hipStreamSynchronize(stream)) != hipSuccess) return dev_err("sync", he);
            if ((he = hipMemcpy(ws + off_tables, tb.data(), tb.size(), hipMemcpyHostToDevice)) != hipSuccess) return dev_err("copy tables", he);
        }
        for (Launch &ln : launches) {
            if (ln.kind == Launch::PASS) {
                PassArgs a = ln.pa;
                a.dst = ws + ln.dst_off;
                a.src = ws + ln.src_off;
                a.slot_path = (const uint64_t *)(ws + off_tables + rp.table_off[ln.level]) + ln.slot_off;
                a.slot_parent = (const uint32_t *)(ws + off_tables + rp.parent_table_off[ln.level]) + ln.slot_off;
                a.prog = (const uint32_t *)(ws + off_blob + ln.plan_off);
                a.prog_words = ln.prog_words;
                a.groups_word = ln.groups_word;
                a.terms_word = ln.terms_word;
                a.slot_parent_base = ln.parent_base;   // parent tables hold level-global indices
                hipEvent_t *e = ev_pair(0);
                if (e) (void)hipEventRecord(e[0], stream);
                if ((he = launch_pass(fp64, ln.R, a, ln.grid, stream)) != hipSuccess) return dev_err("pass", he);
                if (e) (void)hipEventRecord(e[1], stream);
                c.stats.n_sweep_launches++;
                c.stats.sweep_bytes += ln.bytes;
            } else {
                GatherArgs g = ln.ga;
                g.a = ws + ln.dst_off;
                g.b = ws + ln.src_off;
                g.xa = d_xa;
                g.xb = d_xb;
                g.acc = d_acc;
                hipEvent_t *e = ev_pair(1);
                if (e) (void)hipEventRecord(e[0], stream);
                if ((he = launch_gather(fp64, g, stream)) != hipSuccess) return dev_err("gather", he);
                if (e) (void)hipEventRecord(e[1], stream);
                c.stats.n_gather_launches++;
                c.stats.gather_bytes += ln.bytes;
            }
        }
    }
    if (!out_dev && n_bits)
        if ((he = hipMemcpyAsync(amps, d_acc, n_bits * 16, hipMemcpyDeviceToHost, stream)) != hipSuccess) return dev_err("copy amps", he);
    int flag = 0;
    if ((he = hipMemcpyAsync(&flag, d_flag, sizeof(int), hipMemcpyDeviceToHost, stream)) != hipSuccess) return dev_err("copy flag", he);
    if ((he = hipStreamSynchronize(stream)) != hipSuccess) return dev_err("synchronize", he);
    if (flag) { err = "bitstring has bits outside the grid"; return SF_ERR_INVALID; }

    if (timing) {
        for (size_t i = 0; i < ev_cat.size(); ++i) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]);
            if (ev_cat[i] == 0) c.stats.ms_sweep += ms;
            else if (ev_cat[i] == 1) c.stats.ms_gather += ms;
            else c.stats.ms_other += ms;
        }
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    c.stats.n_batches = n_batches * (plain ? n_paths : 1);
    {
        uint64_t pa = 0, pb = 0;
        for (const Launch &ln : launches) if (ln.kind == Launch::PASS) (ln.half ? pb : pa)++;
        c.stats.n_passes_a = pa;
        c.stats.n_passes_b = pb;
    }
    c.stats.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return SF_OK;
}

}  // namespace sf
