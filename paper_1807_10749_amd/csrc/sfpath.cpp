// C ABI entry points (include/sfpath.h).  Every function catches C++
// exceptions and reports errors through return codes and last_error().
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <tuple>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>

#include "jit.hpp"
#include "kernels.hpp"
#include "sf_host.hpp"

using sf::Circuit;


namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int ok()
{
    g_err.clear();
    return SF_OK;
}

template <typename F>
int guarded(F &&f)
{
    try {
        return f();
    } catch (const std::bad_alloc &) {
        return fail(SF_ERR_OOM, "host out of memory");
    } catch (const std::exception &e) {
        return fail(SF_ERR_INVALID, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(SF_ERR_INVALID, "internal error");
    }
}

int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// SplitMix64 (Steele, Lea, Flood 2014).
uint64_t splitmix_next(uint64_t &s)
{
    s += 0x9E3779B97F4A7C15ULL;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int count_crossing(const Circuit &c, uint64_t mask_a)
{
    int k = 0;
    for (const sf_gate_t &g : c.gates)
        if ((g.kind == 4 || g.kind == 5) && (((mask_a >> g.q0) & 1) != ((mask_a >> g.q1) & 1)))
            k += g.kind == 5 ? 2 : 1;   // path bits: two terms for a CZ, four for an iSWAP
    return k;
}

}  // namespace

extern "C" {

const char *last_error(void) { return g_err.c_str(); }

int create_circuit(int rows, int cols, const sf_gate_t *gates, size_t n_gates, sf_circuit_t **out)
{
    return guarded([&]() -> int {
        if (!out) return fail(SF_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (rows < 1 || cols < 1) return fail(SF_ERR_INVALID, "grid must be at least 1 x 1");
        if ((int64_t)rows * cols > 64) return fail(SF_ERR_UNSUPPORTED, "more than 64 qubits");
        if (n_gates && !gates) return fail(SF_ERR_INVALID, "gates is NULL");
        const int n = rows * cols;
        int last_cycle = -1;
        std::vector<int> seen(n, -1);
        for (size_t i = 0; i < n_gates; ++i) {
            const sf_gate_t &g = gates[i];
            if (g.kind > 5) return fail(SF_ERR_INVALID, "gate " + std::to_string(i) + ": unknown kind");
            if (g.q0 >= n) return fail(SF_ERR_INVALID, "gate " + std::to_string(i) + ": qubit outside the grid");
            if (g.cycle < last_cycle) return fail(SF_ERR_INVALID, "gate " + std::to_string(i) + ": cycle decreases");
            last_cycle = g.cycle;
            const bool two = g.kind == 4 || g.kind == 5;
            if (two) {
                if (g.q1 >= n || g.q1 == g.q0)
                    return fail(SF_ERR_INVALID, "gate " + std::to_string(i) + ": bad two-qubit gate qubits");
                const int r0 = g.q0 / cols, c0 = g.q0 % cols, r1 = g.q1 / cols, c1 = g.q1 % cols;
                if (std::abs(r0 - r1) + std::abs(c0 - c1) != 1)
                    return fail(SF_ERR_INVALID, "gate " + std::to_string(i) + ": two-qubit gate on non-adjacent qubits");
            }
            const int qs[2] = {g.q0, two ? (int)g.q1 : -1};
            for (int q : qs) {
                if (q < 0) continue;
                if (seen[q] == g.cycle)
                    return fail(SF_ERR_INVALID, "gate " + std::to_string(i) + ": qubit used twice in one cycle");
                seen[q] = g.cycle;
            }
        }
        sf_circuit *c = new sf_circuit();
        c->rows = rows;
        c->cols = cols;
        c->n = n;
        c->gates.assign(gates, gates + n_gates);
        *out = c;
        return ok();
    });
}

int destroy_circuit(sf_circuit_t *c)
{
    return guarded([&]() -> int {
        if (!c) return ok();
        if (c->dev_ws) (void)hipFree(c->dev_ws);
        for (void *e : c->events) (void)hipEventDestroy((hipEvent_t)e);
        delete c;
        return ok();
    });
}

int set_cut(sf_circuit_t *c, uint64_t mask_a, uint32_t *k_out)
{
    return guarded([&]() -> int {
        if (!c) return fail(SF_ERR_INVALID, "circuit is NULL");
        const uint64_t all = c->n == 64 ? ~uint64_t(0) : ((uint64_t(1) << c->n) - 1);
        if (!(mask_a & 1)) return fail(SF_ERR_INVALID, "block A must hold qubit 0");
        if (mask_a & ~all) return fail(SF_ERR_INVALID, "mask has bits outside the grid");
        if (mask_a == all) return fail(SF_ERR_INVALID, "block B is empty");
        const int qa = popcount64(mask_a), qb = c->n - qa;
        if (qa > 30 || qb > 30) return fail(SF_ERR_UNSUPPORTED, "a block has more than 30 qubits");
        c->mask_a = mask_a;
        c->mask_b = all & ~mask_a;
        c->has_cut = false;
        std::string err;
        const int rc = sf::build_programs(*c, err);
        if (rc) return fail(rc, err);
        c->has_cut = true;
        if (k_out) *k_out = (uint32_t)c->k;
        return ok();
    });
}

int choose_cut(const sf_circuit_t *c, uint64_t *block_a_mask)
{
    return guarded([&]() -> int {
        if (!c || !block_a_mask) return fail(SF_ERR_INVALID, "NULL argument");
        // candidates: (larger block, path bits of the crossing gates, horizontal?, index, mask)
        bool found = false;
        std::tuple<int, int, int, int> best{};
        uint64_t best_mask = 0;
        for (int orient = 0; orient < 2; ++orient) {
            const int lim = orient == 0 ? c->cols - 1 : c->rows - 1;
            for (int i = 0; i < lim; ++i) {
                uint64_t m = 0;
                for (int r = 0; r < c->rows; ++r)
                    for (int col = 0; col < c->cols; ++col)
                        if (orient == 0 ? col <= i : r <= i) m |= uint64_t(1) << (r * c->cols + col);
                const int qa = popcount64(m), qb = c->n - qa;
                auto key = std::make_tuple(std::max(qa, qb), count_crossing(*c, m), orient, i);
                if (!found || key < best) { best = key; best_mask = m; found = true; }
            }
        }
        if (!found) return fail(SF_ERR_UNSUPPORTED, "grid has no straight-line cut");
        if (std::get<0>(best) > 30) return fail(SF_ERR_UNSUPPORTED, "every straight cut leaves a block above 30 qubits");
        *block_a_mask = best_mask;
        return ok();
    });
}

int num_paths(uint32_t k, double f, uint64_t *n_out)
{
    if (!n_out) return fail(SF_ERR_INVALID, "n_out is NULL");
    if (k > 62) return fail(SF_ERR_UNSUPPORTED, "k > 62");
    if (!(f > 0.0) || f > 1.0) return fail(SF_ERR_INVALID, "f must lie in (0, 1]");
    *n_out = (uint64_t)std::ceil(std::ldexp(f, (int)k));
    return ok();
}

int sample_paths(uint32_t k, double f, uint64_t seed, uint64_t *out, uint64_t cap, uint64_t *n_out)
{
    return guarded([&]() -> int {
        uint64_t m = 0;
        int rc = num_paths(k, f, &m);
        if (rc) return rc;
        if (!out || m > cap) return fail(SF_ERR_INVALID, "output array too small");
        const uint64_t N = uint64_t(1) << k;
        std::unordered_set<uint64_t> chosen;
        chosen.reserve((size_t)m * 2);
        uint64_t s = seed, filled = 0;
        for (uint64_t j = N - m; j < N; ++j) {
            const uint64_t r = splitmix_next(s);
            const uint64_t t = (uint64_t)(((unsigned __int128)r * (unsigned __int128)(j + 1)) >> 64);
            const uint64_t pick = chosen.insert(t).second ? t : j;
            if (pick == j) chosen.insert(j);
            out[filled++] = pick;
        }
        std::sort(out, out + m);
        if (n_out) *n_out = m;
        return ok();
    });
}

int workspace_size(const sf_circuit_t *c, uint64_t n_paths, size_t n_bits, uint32_t flags, size_t *bytes)
{
    return guarded([&]() -> int {
        if (!c || !bytes) return fail(SF_ERR_INVALID, "NULL argument");
        if (!c->has_cut) return fail(SF_ERR_NO_CUT, "set_cut has not been called");
        return sf::estimate_workspace(*c, n_paths, n_bits, flags, bytes) ? fail(SF_ERR_INVALID, "estimate failed") : ok();
    });
}

namespace {
// Argument rules shared by run_paths and autotune (both end in sf::execute); 0 or an error code
// with the thread's message set.  The device sort, select and reduce of the bitstrings count in
// int, hence the INT_MAX limit.
int check_run_args(const sf_circuit_t *c, const uint64_t *bitstrings, size_t n_bits, const double *amps,
                   uint32_t flags, const void *workspace, size_t workspace_bytes)
{
    if (!c) return fail(SF_ERR_INVALID, "circuit is NULL");
    if (!c->has_cut) return fail(SF_ERR_NO_CUT, "set_cut has not been called");
    if (n_bits && (!bitstrings || !amps)) return fail(SF_ERR_INVALID, "bitstrings or amps is NULL");
    if (flags & ~uint32_t(63)) return fail(SF_ERR_INVALID, "unknown flag");
    if (workspace && workspace_bytes < (size_t(1) << 28)) return fail(SF_ERR_OOM, "workspace smaller than 256 MiB");
    if (n_bits > (size_t)INT_MAX) return fail(SF_ERR_UNSUPPORTED, "more than 2^31 - 1 bitstrings");
    return SF_OK;
}
}  // namespace

}  // extern "C"

namespace sf {
// run_paths on a workspace of the caller's choosing that may be smaller than run_paths'
// 256 MiB minimum (the executor still refuses one that cannot hold a single slot per level).
int run_paths_in(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
                 const uint64_t *bitstrings, size_t n_bits, double *amps, uint32_t flags, void *hip_stream,
                 void *workspace, size_t workspace_bytes)
{
    return guarded([&]() -> int {
        if (const int rc = check_run_args(c, bitstrings, n_bits, amps, flags, nullptr, 0)) return rc;
        std::string err;
        const int rc = sf::execute(*c, path_ids, path_begin, n_paths, bitstrings, n_bits, amps, flags, hip_stream,
                                   workspace, workspace_bytes, err, false, true);
        return rc ? fail(rc, err) : ok();
    });
}

int set_error(int code, const std::string &msg) { return fail(code, msg); }
}  // namespace sf

extern "C" {

int run_paths(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
              const uint64_t *bitstrings, size_t n_bits, double *amps, uint32_t flags, void *hip_stream,
              void *workspace, size_t workspace_bytes)
{
    return guarded([&]() -> int {
        if (const int rc = check_run_args(c, bitstrings, n_bits, amps, flags, workspace, workspace_bytes)) return rc;
        std::string err;
        const int rc = sf::execute(*c, path_ids, path_begin, n_paths, bitstrings, n_bits, amps, flags, hip_stream,
                                   workspace, workspace_bytes, err);
        return rc ? fail(rc, err) : ok();
    });
}

int set_tuning(sf_circuit_t *c, const sf_tuning_t *t)
{
    if (!c || !t) return fail(SF_ERR_INVALID, "NULL argument");
    if (t->reg_qubits > 5) return fail(SF_ERR_INVALID, "reg_qubits must be at most 5");
    if (t->dense_qubits == 1 || t->dense_qubits > 4) return fail(SF_ERR_INVALID, "dense_qubits must be 0 or 2..4");
    if (t->no_leaf_fold > 1) return fail(SF_ERR_INVALID, "no_leaf_fold must be 0 or 1");
    if (t->fold_levels > 62) return fail(SF_ERR_INVALID, "fold_levels must be at most 62");
    if (t->chain_passes > 1) return fail(SF_ERR_INVALID, "chain_passes must be 0 or 1");
    if (t->no_row_skip > 1) return fail(SF_ERR_INVALID, "no_row_skip must be 0 or 1");
    if (t->no_defer > 1) return fail(SF_ERR_INVALID, "no_defer must be 0 or 1");
    if (t->no_chain_merge > 1) return fail(SF_ERR_INVALID, "no_chain_merge must be 0 or 1");
    if (t->jit > 1) return fail(SF_ERR_INVALID, "jit must be 0 or 1");
    if (t->no_tail_move > 1) return fail(SF_ERR_INVALID, "no_tail_move must be 0 or 1");
    auto pow2ok = [](uint32_t v) { return v == 0 || (v & (v - 1)) == 0; };
    if (!pow2ok(t->leaf_batch) || !pow2ok(t->max_slots)) return fail(SF_ERR_INVALID, "batch sizes must be powers of two");
    c->tuning = *t;
    c->plan_cache.clear();
    return ok();
}

int get_tuning(const sf_circuit_t *c, sf_tuning_t *t)
{
    if (!c || !t) return fail(SF_ERR_INVALID, "NULL argument");
    *t = c->tuning;
    return ok();
}

namespace {
std::mutex g_tune_mu;
std::map<std::string, sf_tuning_t> g_tune_cache;

// "<arch>:<compute units>" of the current device: tunings are kept per device kind.
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
    return arch + ":" + std::to_string(prop.multiProcessorCount);
}

// Effective rates of the cost model (bytes/s, s per launch) on one MI355X, from
// measured pass and gather kernels; only the ranking of candidates depends on them.
constexpr double kSweepRate = 5.0e12, kGatherRate = 6.0e12, kLaunchCost = 4e-6;
}  // namespace

int autotune(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
             const uint64_t *bitstrings, size_t n_bits, double *amps, uint32_t flags, void *hip_stream,
             void *workspace, size_t workspace_bytes, uint32_t n_measure, sf_tuning_t *best)
{
    return guarded([&]() -> int {
        if (!best) return fail(SF_ERR_INVALID, "best is NULL");
        if (const int rc = check_run_args(c, bitstrings, n_bits, amps, flags, workspace, workspace_bytes)) return rc;
        if (flags & SF_ACCUMULATE) return fail(SF_ERR_INVALID, "autotune overwrites amps: SF_ACCUMULATE is not accepted");
        const bool fp64 = (flags & SF_FP64_SWEEPS) != 0;
        const std::string key = device_tag() + "/" + std::to_string(c->half[0].q) + "/" + std::to_string(c->half[1].q) + "/" +
                                std::to_string(c->k) + "/" + std::to_string(c->levels.size()) + "/" +
                                std::to_string(n_paths) + "/" + std::to_string(n_bits) + "/" +
                                std::to_string(flags & (SF_FP64_SWEEPS | SF_PLAIN));
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                c->tuning = it->second;
                *best = it->second;
                return ok();
            }
        }
        const sf_tuning_t start = c->tuning;
        std::vector<sf_tuning_t> cands;
        const uint32_t regs[3] = {fp64 ? 4u : 5u, fp64 ? 3u : 4u, fp64 ? 2u : 3u};
        const uint32_t leafs[4] = {0u, 4096u, 1024u, 256u};
        const uint32_t wpcs[3] = {128u, 32u, 64u};
        sf_tuning_t probe = c->tuning;
        probe.no_leaf_fold = 0;
        probe.fold_levels = 0;
        std::swap(probe, c->tuning);
        const int max_fold = sf::fold_depth(*c);
        std::swap(probe, c->tuning);
        for (uint32_t r : regs)
            for (uint32_t w : wpcs)
                for (uint32_t dq : {0u, 2u, 3u, 4u}) {
                    if (dq && fp64) continue;                 // dense blocks on matrix cores: complex64 only
                    for (int F = 1; F <= max_fold; ++F) {     // F trailing levels folded into the gather
                        const int Fp = max_fold > 1 ? max_fold - 1 : 1;
                        if (F != max_fold && F != Fp) continue;
                        cands.push_back(sf_tuning_t{r, 0, 0, w, dq, 0, (uint32_t)F, start.chain_passes, start.no_row_skip, start.no_defer, start.no_chain_merge, 0, start.no_tail_move});
                    }
                    for (uint32_t lf : leafs) cands.push_back(sf_tuning_t{r, lf, 0, w, dq, 1, 0, start.chain_passes, start.no_row_skip, start.no_defer, start.no_chain_merge, 0, start.no_tail_move});
                }
        // rank by the planned cost
        std::vector<std::pair<double, size_t>> ranked;
        for (size_t i = 0; i < cands.size(); ++i) {
            c->tuning = cands[i];
            std::string err;
            if (sf::execute(*c, path_ids, path_begin, n_paths, bitstrings, n_bits, amps, flags, hip_stream, workspace,
                            workspace_bytes, err, true))
                continue;
            const sf_run_stats_t &st = c->stats;
            const double model = (double)st.sweep_bytes / kSweepRate + (double)st.gather_bytes / kGatherRate +
                                 (double)(st.n_sweep_launches + st.n_gather_launches) * kLaunchCost;
            ranked.push_back({model, i});
        }
        if (ranked.empty()) { c->tuning = start; return fail(SF_ERR_UNSUPPORTED, "no tuning candidate could be planned"); }
        std::sort(ranked.begin(), ranked.end());
        // time the best-ranked candidate of every kind (leaf handling x dense blocks) first, since
        // the model compares kinds less reliably than tunings of one kind; then fill by rank
        std::vector<sf_tuning_t> measure;
        measure.push_back(start);
        std::vector<size_t> picked;
        std::set<std::tuple<uint32_t, uint32_t, uint32_t>> kinds;
        for (size_t i = 0; i < ranked.size(); ++i) {
            const sf_tuning_t &t = cands[ranked[i].second];
            if (kinds.insert({t.no_leaf_fold, t.fold_levels, t.dense_qubits}).second) picked.push_back(i);
        }
        for (size_t i = 0; i < ranked.size() && picked.size() < (size_t)std::max(1u, n_measure); ++i)
            if (std::find(picked.begin(), picked.end(), i) == picked.end()) picked.push_back(i);
        std::sort(picked.begin(), picked.end());
        for (size_t i : picked) measure.push_back(cands[ranked[i].second]);
        double best_t = 1e300;
        sf_tuning_t best_t_cfg = start;
        // candidates are timed with interpreted passes (compiling every candidate's programs would
        // cost seconds each); the winner keeps the caller's jit setting
        for (const sf_tuning_t &t : measure) {
            c->tuning = t;
            c->tuning.jit = 0;
            double tmin = 1e300;
            for (int rep = 0; rep < 2; ++rep) {
                std::string err;
                const auto t0 = std::chrono::steady_clock::now();
                const int rc = sf::execute(*c, path_ids, path_begin, n_paths, bitstrings, n_bits, amps, flags, hip_stream,
                                           workspace, workspace_bytes, err);
                if (rc) { c->tuning = start; return fail(rc, err); }
                tmin = std::min(tmin, std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
            }
            if (tmin < best_t) { best_t = tmin; best_t_cfg = t; }
        }
        best_t_cfg.jit = start.jit;
        c->tuning = best_t_cfg;
        *best = best_t_cfg;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best_t_cfg;
        return ok();
    });
}

int save_tuning_cache(const char *path)
{
    return guarded([&]() -> int {
        if (!path) return fail(SF_ERR_INVALID, "path is NULL");
        std::lock_guard<std::mutex> lk(g_tune_mu);
        FILE *f = std::fopen(path, "w");
        if (!f) return fail(SF_ERR_INVALID, std::string("cannot write ") + path);
        std::fprintf(f, "# sfpath tuning cache: key reg_qubits leaf_batch max_slots waves_per_cu dense_qubits "
                        "no_leaf_fold fold_levels chain_passes no_row_skip no_defer no_chain_merge jit no_tail_move\n");
        for (const auto &kv : g_tune_cache) {
            const sf_tuning_t &t = kv.second;
            std::fprintf(f, "%s %u %u %u %u %u %u %u %u %u %u %u %u %u\n", kv.first.c_str(), t.reg_qubits, t.leaf_batch,
                         t.max_slots, t.waves_per_cu, t.dense_qubits, t.no_leaf_fold, t.fold_levels, t.chain_passes,
                         t.no_row_skip, t.no_defer, t.no_chain_merge, t.jit, t.no_tail_move);
        }
        const bool bad = std::ferror(f) != 0;
        if (std::fclose(f) != 0 || bad) return fail(SF_ERR_INVALID, std::string("cannot write ") + path);
        return ok();
    });
}

int load_tuning_cache(const char *path, uint32_t *n_loaded)
{
    return guarded([&]() -> int {
        if (!path) return fail(SF_ERR_INVALID, "path is NULL");
        FILE *f = std::fopen(path, "r");
        if (!f) return fail(SF_ERR_INVALID, std::string("cannot read ") + path);
        std::map<std::string, sf_tuning_t> got;
        char line[1024];
        int lineno = 0;
        while (std::fgets(line, sizeof(line), f)) {
            ++lineno;
            if (line[0] == '#' || line[0] == '\n') continue;
            char key[512];
            sf_tuning_t t{};
            char extra;
            // entries written before chain_passes / no_row_skip / no_defer / no_chain_merge / jit /
            // no_tail_move existed have fields less (read as 0)
            const int got_n = std::sscanf(line, "%511s %u %u %u %u %u %u %u %u %u %u %u %u %u %c", key, &t.reg_qubits,
                                          &t.leaf_batch, &t.max_slots, &t.waves_per_cu, &t.dense_qubits,
                                          &t.no_leaf_fold, &t.fold_levels, &t.chain_passes, &t.no_row_skip,
                                          &t.no_defer, &t.no_chain_merge, &t.jit, &t.no_tail_move, &extra);
            if (got_n < 8 || got_n > 14 || t.reg_qubits > 5 || t.dense_qubits == 1 || t.dense_qubits > 4 ||
                t.no_leaf_fold > 1 || t.fold_levels > 62 || t.chain_passes > 1 || t.no_row_skip > 1 ||
                t.no_defer > 1 || t.no_chain_merge > 1 || t.jit > 1 || t.no_tail_move > 1) {
                std::fclose(f);
                return fail(SF_ERR_INVALID, std::string(path) + ":" + std::to_string(lineno) + ": malformed entry");
            }
            got[key] = t;
        }
        std::fclose(f);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto &kv : got) g_tune_cache[kv.first] = kv.second;
        if (n_loaded) *n_loaded = (uint32_t)got.size();
        return ok();
    });
}

int get_run_stats(const sf_circuit_t *c, sf_run_stats_t *s)
{
    if (!c || !s) return fail(SF_ERR_INVALID, "NULL argument");
    *s = c->stats;
    return ok();
}

int describe_plan(sf_circuit_t *c, char *out, size_t cap)
{
    return guarded([&]() -> int {
        if (!c || !out || !cap) return fail(SF_ERR_INVALID, "NULL argument");
        if (!c->has_cut) return fail(SF_ERR_NO_CUT, "set_cut has not been called");
        std::string s;
        const int R = c->tuning.reg_qubits ? (int)c->tuning.reg_qubits : 5;
        const int L = (int)c->levels.size() - 1;
        s += "k=" + std::to_string(c->k) + " qA=" + std::to_string(c->half[0].q) +
             " qB=" + std::to_string(c->half[1].q) + " levels=" + std::to_string(L) + "\n";
        // pairs of path bits that must agree for a nonzero term (other paths are skipped)
        s += "equal path bits:";
        for (const auto &pr : c->equal_bits) s += " " + std::to_string(pr.first) + "=" + std::to_string(pr.second);
        s += "\n";
        for (int l = 0; l <= L; ++l) {
            int p = std::min(c->levels[l].bits_after, 20);
            const int qmin = std::min(c->half[0].q, c->half[1].q);
            if (qmin + p < 6) p = 6 - qmin;
            s += "level " + std::to_string(l) + " cycle " + std::to_string(c->levels[l].cycle) +
                 " bits " + std::to_string(c->levels[l].bits_after) + " p " + std::to_string(p) + ":";
            const int FD = sf::fold_depth(*c);
            if (FD && l > L - FD) {
                const sf::LeafFold &f0 = c->half[0].folds[FD - 1], &f1 = c->half[1].folds[FD - 1];
                s += " A " + std::to_string(c->half[0].segments[l].size()) + " ops, B " +
                     std::to_string(c->half[1].segments[l].size()) + " ops folded into the gather";
                if (l == L && sf::fold_general(*c, FD))
                    s += " (" + std::to_string(FD) + " levels, branch bits " + std::to_string(f0.nb) +
                         ", general form; A: S' " + std::to_string(f0.g_ns) + " qubits, T' " +
                         std::to_string(f0.g_nt) + "; B: S' " + std::to_string(f1.g_ns) + " qubits, T' " +
                         std::to_string(f1.g_nt) + "; used when cheaper than writing the levels)";
                else if (l == L)
                    s += " (" + std::to_string(FD) + " levels, branch bits " + std::to_string(f0.nb) +
                         (f0.iswap ? ", " + std::to_string(f0.ng) + " iSWAP gates" : std::string()) + "; A: S " +
                         std::to_string(f0.n_s) + " qubits, T " + std::to_string(f0.n_t) + "; B: S " +
                         std::to_string(f1.n_s) + " qubits, T " + std::to_string(f1.n_t) + ")";
                s += "\n";
                continue;
            }
            for (int h = 0; h < 2; ++h) {
                const sf::SegmentPlan &sp = sf::get_segment_plan(*c, h, l, p, R, (int)c->tuning.dense_qubits);
                int nd = 0;
                for (const sf::HalfOp &op : c->half[h].segments[l]) nd += sf::is_diag(op.kind) ? 0 : 1;
                s += std::string(h ? "  B " : " A ") + std::to_string(c->half[h].segments[l].size()) + " ops (" +
                     std::to_string(nd) + " non-diag) " + std::to_string(sp.passes.size()) + " passes [";
                for (size_t i = 0; i < sp.passes.size(); ++i) {
                    // zN: the pass reads a source whose zero subspace spans N projected qubits
                    uint64_t zq = 0;
                    for (const auto &e : sp.passes[i].zero_in) zq |= uint64_t(1) << e.first;
                    // gates on register qubits (r) and on lane qubits (l, lane shuffles)
                    int n_lane = 0;
                    for (const sf::PassOp &op : sp.passes[i].ops) n_lane += op.type == sf::PO_LANE ? 1 : 0;
                    s += (i ? "," : "") + std::to_string(sp.passes[i].n_nondiag) + "g" +
                         (n_lane ? "(" + std::to_string(n_lane) + "l)" : std::string()) + "/" +
                         (sp.passes[i].dense ? std::string("dense") : std::to_string(sp.passes[i].groups.size()) + "d") +
                         (zq ? "/z" + std::to_string(__builtin_popcountll(zq)) : std::string());
                }
                s += "]";
                // qubits of the level's non-diagonal gates and of its branch operators
                uint64_t ndq = 0, brq = 0;
                for (const sf::HalfOp &op : c->half[h].segments[l]) {
                    if (sf::is_branch(op.kind)) brq |= uint64_t(1) << op.q0;
                    else if (!sf::is_diag(op.kind)) {
                        ndq |= uint64_t(1) << op.q0;
                        if (sf::is_two_qubit(op.kind)) ndq |= uint64_t(1) << op.q1;
                    }
                }
                char qb[64];
                std::snprintf(qb, sizeof qb, "{nd 0x%llx br 0x%llx}", (unsigned long long)ndq, (unsigned long long)brq);
                s += qb;
            }
            s += "\n";
            // the level the path sum reads: qubits inside a tile of each block's last pass, and
            // the qubits whose rows the path sum varies (row masks skip the other tiles)
            const int FDr = sf::fold_depth(*c);
            if (l == L - FDr) {
                s += "  path-sum reads this level:";
                for (int h = 0; h < 2; ++h) {
                    const sf::SegmentPlan &sp = sf::get_segment_plan(*c, h, l, p, R, (int)c->tuning.dense_qubits);
                    uint32_t inside = 0;
                    if (!sp.passes.empty() && !sp.passes.back().dense) {
                        const sf::PassPlan &pp = sp.passes.back();
                        for (int k = 0; k < pp.R; ++k) inside |= 1u << (pp.reg_pos[k] - p);
                        const int lane_bits = pp.lane_q4 >= 0 ? 4 : pp.lane_q >= 0 ? 5 : 6;
                        if (lane_bits > p) inside |= (1u << (lane_bits - p)) - 1u;
                        if (pp.lane_q >= 0) inside |= 1u << pp.lane_q;
                        if (pp.lane_q4 >= 0) inside |= 1u << pp.lane_q4;
                    }
                    uint32_t vary = 0;
                    if (FDr) {
                        const sf::LeafFold &f = c->half[h].folds[FDr - 1];
                        vary = sf::fold_general(*c, FDr) ? f.g_smask : f.iswap ? f.qmask : f.smask;
                    }
                    char buf[96];
                    std::snprintf(buf, sizeof buf, " %s tile qubits 0x%x, rows vary 0x%x (%d outside);", h ? "B" : "A",
                                  inside, vary, __builtin_popcount(vary & ~inside));
                    s += buf;
                    if (h == 0 && FDr == 1 && sf::fold_general(*c, FDr) && !c->tuning.no_defer) {
                        const sf::DeferredLevel d = sf::deferred_level(*c, 0, l);
                        if (d.ok && !(d.mask & vary)) {
                            std::snprintf(buf, sizeof buf, " A deferred (projected qubits 0x%x);", d.mask);
                            s += buf;
                        }
                    }
                }
                s += "\n";
            }
        }
        std::strncpy(out, s.c_str(), cap - 1);
        out[cap - 1] = 0;
        return ok();
    });
}


// ------------------------------------------------------------------ rejection sampling
// Section "Frugal rejection sampling" and its figure: Algorithm 1 (basic) and Algorithm 2
// (frugal) turn a batch of output probabilities of uniformly drawn candidates into samples.

int rejection_m(uint32_t n_qubits, double eps, uint32_t flags, double *m)
{
    if (!m) return fail(SF_ERR_INVALID, "m is NULL");
    if (n_qubits < 1 || n_qubits > 64 || !(eps > 0.0) || !(eps < 1.0)) return fail(SF_ERR_INVALID, "bad n_qubits or eps");
    if (flags & ~uint32_t(SF_SAMPLE_BASIC)) return fail(SF_ERR_INVALID, "unknown flag");
    if (flags & SF_SAMPLE_BASIC) {
        *m = std::ceil(n_qubits * std::log(2.0) - std::log(eps));     // M = ceil(ln(N / eps))
    } else {
        int mp = 1;                                                     // e^{-M'} (1 + M') <= eps
        while (std::exp(-(double)mp) * (1.0 + mp) > eps) ++mp;
        *m = mp;
    }
    return ok();
}

int sample_bitstrings(uint32_t n_qubits, uint64_t count, uint64_t seed, uint64_t *out)
{
    return guarded([&]() -> int {
        if (count && !out) return fail(SF_ERR_INVALID, "out is NULL");
        if (n_qubits < 1 || n_qubits > 64) return fail(SF_ERR_INVALID, "n_qubits must be 1..64");
        if (n_qubits < 64 && count > (uint64_t(1) << n_qubits)) return fail(SF_ERR_INVALID, "more bitstrings than exist");
        const uint64_t mask = n_qubits == 64 ? ~uint64_t(0) : ((uint64_t(1) << n_qubits) - 1);
        // open-addressing set of the values drawn so far (value + 1 stored, 0 = empty), at most
        // half full; hashed with a Fibonacci multiplier so consecutive values spread out
        uint64_t cap = 16;
        while (cap < 2 * count) cap <<= 1;
        std::vector<uint64_t> slot(cap, 0);
        const int shift = 64 - __builtin_ctzll(cap);
        uint64_t st = seed, got = 0;
        while (got < count) {
            const uint64_t x = splitmix_next(st) & mask;
            uint64_t i = (x * 0x9E3779B97F4A7C15ULL) >> shift;
            while (slot[i] && slot[i] != x + 1) i = (i + 1) & (cap - 1);
            if (!slot[i]) {
                slot[i] = x + 1;
                out[got++] = x;
            }
        }
        return ok();
    });
}

int rejection_workspace_size(uint64_t n, size_t *bytes)
{
    return guarded([&]() -> int {
        if (!bytes) return fail(SF_ERR_INVALID, "bytes is NULL");
        if (n > (uint64_t(1) << 31)) return fail(SF_ERR_UNSUPPORTED, "more than 2^31 candidates");
        size_t temp = 0;
        hipError_t e = sf::reject_temp_bytes(std::max<uint64_t>(n, 1), &temp);
        if (e != hipSuccess) return fail(SF_ERR_DEVICE, std::string("temp size: ") + hipGetErrorString(e));
        auto al = [](size_t x) { return (x + 255) / 256 * 256; };
        *bytes = al(n) + al(n * 8) + 256 + al(temp);
        return ok();
    });
}

int rejection_accept(const double *amps, uint64_t n, uint32_t n_qubits, double m, uint64_t seed, uint32_t flags,
                     uint32_t *accepted, uint64_t *n_accepted, double *err_est, void *hip_stream,
                     void *workspace, size_t workspace_bytes)
{
    return guarded([&]() -> int {
        if (!n_accepted || !err_est) return fail(SF_ERR_INVALID, "NULL argument");
        if (n && (!amps || !accepted || !workspace)) return fail(SF_ERR_INVALID, "NULL device buffer");
        if (n_qubits < 1 || n_qubits > 64 || !(m > 0.0)) return fail(SF_ERR_INVALID, "bad n_qubits or m");
        if (flags & ~uint32_t(SF_SAMPLE_BASIC)) return fail(SF_ERR_INVALID, "unknown flag");
        if (n > (uint64_t)INT_MAX) return fail(SF_ERR_UNSUPPORTED, "more than 2^31 - 1 candidates");
        size_t need = 0;
        int rc = rejection_workspace_size(n, &need);
        if (rc) return rc;
        if (n && workspace_bytes < need) return fail(SF_ERR_OOM, "workspace too small");
        *n_accepted = 0;
        *err_est = 0.0;
        if (!n) return ok();
        hipStream_t s = (hipStream_t)hip_stream;
        auto al = [](size_t x) { return (x + 255) / 256 * 256; };
        char *w = (char *)workspace;
        uint8_t *flag = (uint8_t *)w;
        double *excess = (double *)(w + al(n));
        uint64_t *d_count = (uint64_t *)(w + al(n) + al(n * 8));
        double *d_sum = (double *)(w + al(n) + al(n * 8) + 8);
        char *temp = w + al(n) + al(n * 8) + 256;
        const size_t temp_bytes = workspace_bytes - (al(n) + al(n * 8) + 256);
        const double scale = std::ldexp(1.0, (int)n_qubits) / m;        // t = p N / M
        hipError_t e = sf::launch_accept(amps, n, scale, seed, (flags & SF_SAMPLE_BASIC) ? 1 : 0, flag, excess,
                                         accepted, d_count, d_sum, temp, temp_bytes, s);
        if (e != hipSuccess) return fail(SF_ERR_DEVICE, std::string("accept: ") + hipGetErrorString(e));
        uint64_t cnt = 0;
        double sum = 0.0;
        if ((e = hipMemcpyAsync(&cnt, d_count, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(&sum, d_sum, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail(SF_ERR_DEVICE, std::string("accept: ") + hipGetErrorString(e));
        *n_accepted = cnt;
        *err_est = sum * std::ldexp(1.0, (int)n_qubits) / (double)n;   // (N / n) sum_{t > 1} p
        return ok();
    });
}

int frugal_sample(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
                  uint64_t n_candidates, double m, uint64_t seed_candidates, uint64_t seed_accept, uint32_t flags,
                  void *hip_stream, void *workspace, size_t workspace_bytes, uint64_t *out, uint64_t *n_out,
                  double *err_est)
{
    return guarded([&]() -> int {
        if (!c || !n_out || !err_est) return fail(SF_ERR_INVALID, "NULL argument");
        if (n_candidates && !out) return fail(SF_ERR_INVALID, "out is NULL");
        if (!c->has_cut) return fail(SF_ERR_NO_CUT, "set_cut has not been called");
        const uint32_t run_flags = flags & (SF_FP64_SWEEPS | SF_PLAIN);
        if (flags & ~uint32_t(SF_FP64_SWEEPS | SF_PLAIN | SF_SAMPLE_BASIC)) return fail(SF_ERR_INVALID, "unknown flag");
        if (n_candidates > (uint64_t)INT_MAX) return fail(SF_ERR_UNSUPPORTED, "more than 2^31 - 1 candidates");
        *n_out = 0;
        *err_est = 0.0;
        // Step 2: candidates
        std::vector<uint64_t> cand(n_candidates);
        int rc = sample_bitstrings((uint32_t)c->n, n_candidates, seed_candidates, cand.data());
        if (rc) return rc;
        if (!n_candidates) return ok();
        size_t rws = 0;
        if ((rc = rejection_workspace_size(n_candidates, &rws))) return rc;
        auto al = [](size_t x) { return (x + 255) / 256 * 256; };
        const size_t own = al(n_candidates * 8) + al(n_candidates * 16) + al(n_candidates * 4) + al(rws);
        // device arrays: carved from the end of the caller's workspace, else allocated here
        char *base = nullptr;
        void *run_ws = nullptr;
        size_t run_ws_bytes = 0;
        bool allocated = false;
        hipError_t e;
        if (workspace) {
            if (workspace_bytes < own + (size_t(1) << 28)) return fail(SF_ERR_OOM, "workspace too small");
            base = (char *)workspace + (workspace_bytes - own) / 256 * 256;
            run_ws = workspace;
            run_ws_bytes = (size_t)(base - (char *)workspace);
        } else {
            if ((e = hipMalloc((void **)&base, own)) != hipSuccess) return fail(SF_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
            allocated = true;
        }
        uint64_t *d_bits = (uint64_t *)base;
        double *d_amps = (double *)(base + al(n_candidates * 8));
        uint32_t *d_acc = (uint32_t *)(base + al(n_candidates * 8) + al(n_candidates * 16));
        char *d_rws = base + al(n_candidates * 8) + al(n_candidates * 16) + al(n_candidates * 4);
        hipStream_t s = (hipStream_t)hip_stream;
        auto finish = [&](int code) {
            if (allocated) { (void)hipStreamSynchronize(s); (void)hipFree(base); }
            return code;
        };
        if ((e = hipMemcpyAsync(d_bits, cand.data(), n_candidates * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
            return finish(fail(SF_ERR_DEVICE, std::string("copy candidates: ") + hipGetErrorString(e)));
        // Step 3: their probabilities at once
        rc = run_paths(c, path_ids, path_begin, n_paths, d_bits, n_candidates, d_amps,
                       run_flags | SF_BITS_ON_DEVICE | SF_OUT_ON_DEVICE, hip_stream, run_ws, run_ws_bytes);
        if (rc) return finish(rc);
        // Step 4: acceptance
        uint64_t n_acc = 0;
        rc = rejection_accept(d_amps, n_candidates, (uint32_t)c->n, m, seed_accept, flags & SF_SAMPLE_BASIC, d_acc,
                              &n_acc, err_est, hip_stream, d_rws, rws);
        if (rc) return finish(rc);
        std::vector<uint32_t> idx(n_acc);
        if (n_acc && (e = hipMemcpy(idx.data(), d_acc, n_acc * 4, hipMemcpyDeviceToHost)) != hipSuccess)
            return finish(fail(SF_ERR_DEVICE, std::string("copy accepted: ") + hipGetErrorString(e)));
        for (uint64_t i = 0; i < n_acc; ++i) out[i] = cand[idx[i]];
        *n_out = n_acc;
        return finish(ok());
    });
}


// ------------------------------------------------------------------ validation of results
// Appendix on validating simulation results: state overlap from amplitudes at common indices
// and the Verifier's side of the two-party protocol; linear cross-entropy fidelity.

namespace {
// sums[0..3] = Re, Im of sum conj(a) b, sum |a|^2, sum |b|^2; partial sums per block are added
// on the host in block order
int overlap_sums(const double *a, const double *b, uint64_t n, hipStream_t s, double sums[4])
{
    for (int q = 0; q < 4; ++q) sums[q] = 0.0;
    if (!n) return SF_OK;
    const unsigned blocks = (unsigned)std::min<uint64_t>(1024, (n + 255) / 256);
    double *partial = nullptr;
    hipError_t e = hipMallocAsync((void **)&partial, (size_t)blocks * 32, s);
    if (e != hipSuccess) return fail(SF_ERR_OOM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    std::vector<double> h((size_t)blocks * 4);
    if ((e = sf::launch_overlap(a, b, n, partial, blocks, s)) != hipSuccess ||
        (e = hipMemcpyAsync(h.data(), partial, h.size() * 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipFreeAsync(partial, s)) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
        return fail(SF_ERR_DEVICE, std::string("overlap: ") + hipGetErrorString(e));
    for (unsigned i = 0; i < blocks; ++i)
        for (int q = 0; q < 4; ++q) sums[q] += h[4 * (size_t)i + q];
    return SF_OK;
}
}  // namespace

int fidelity_estimate(const double *a, const double *b, uint64_t n, void *hip_stream, double *f_e, double *norm_a,
                      double *norm_b)
{
    return guarded([&]() -> int {
        if (!f_e) return fail(SF_ERR_INVALID, "f_e is NULL");
        if (n && (!a || !b)) return fail(SF_ERR_INVALID, "NULL device array");
        double sm[4];
        const int rc = overlap_sums(a, b, n, (hipStream_t)hip_stream, sm);
        if (rc) return rc;
        *f_e = (sm[2] > 0.0 && sm[3] > 0.0) ? (sm[0] * sm[0] + sm[1] * sm[1]) / (sm[2] * sm[3]) : 0.0;
        if (norm_a) *norm_a = sm[2];
        if (norm_b) *norm_b = sm[3];
        return ok();
    });
}

int xeb_fidelity(const double *amps, uint64_t n, uint32_t n_qubits, void *hip_stream, double *f)
{
    return guarded([&]() -> int {
        if (!f) return fail(SF_ERR_INVALID, "f is NULL");
        if (n && !amps) return fail(SF_ERR_INVALID, "NULL device array");
        if (n_qubits < 1 || n_qubits > 64) return fail(SF_ERR_INVALID, "n_qubits must be 1..64");
        double sm[4];
        const int rc = overlap_sums(amps, nullptr, n, (hipStream_t)hip_stream, sm);
        if (rc) return rc;
        *f = n ? std::ldexp(sm[2], (int)n_qubits) / (double)n - 1.0 : 0.0;   // N <p(x)> - 1
        return ok();
    });
}

int compile_segment_kernels(sf_circuit_t *c, int half, uint32_t first_level, uint32_t last_level,
                            uint32_t slot_bits, uint32_t reg_qubits, uint32_t fp64, uint32_t *n_kernels,
                            uint64_t *code_bytes)
{
    return guarded([&]() -> int {
        if (!c || !n_kernels || !code_bytes) return fail(SF_ERR_INVALID, "NULL argument");
        if (!c->has_cut) return fail(SF_ERR_NO_CUT, "set_cut has not been called");
        if (half < 0 || half > 1) return fail(SF_ERR_INVALID, "half must be 0 or 1");
        const uint32_t L = (uint32_t)c->levels.size() - 1;
        if (first_level > last_level || last_level > L) return fail(SF_ERR_INVALID, "levels out of range");
        if (reg_qubits < 1 || reg_qubits > (fp64 ? 4u : 5u)) return fail(SF_ERR_INVALID, "reg_qubits out of range");
        if (slot_bits > 24) return fail(SF_ERR_INVALID, "slot_bits must be at most 24");
        const sf::SegmentPlan &sp = sf::get_segment_plan_range(*c, half, (int)first_level, (int)last_level,
                                                               (int)slot_bits, (int)reg_qubits, 0);
        if (!sp.ok) return fail(SF_ERR_UNSUPPORTED, "the segment could not be planned");
        std::vector<std::string> srcs;
        for (const sf::PassPlan &pp : sp.passes) {
            const std::string prog = sf::jit_program(pp);
            if (prog.empty()) continue;
            const bool z = !pp.zero_in.empty() && !fp64 && (pp.R == 4 || pp.R == 5);
            srcs.push_back(sf::jit_kernel(fp64 != 0, pp.R, prog, z, 0, std::string(), false));
        }
        std::string err;
        if (int rc = sf::jit_compile_only(srcs, "gfx950", code_bytes, err)) return fail(rc, err);
        *n_kernels = (uint32_t)srcs.size();
        return ok();
    });
}

int read_bandwidth(const void *buf, size_t bytes, uint32_t reps, uint32_t grid, void *hip_stream, double *ms_out)
{
    return guarded([&]() -> int {
        if (!buf || !ms_out) return fail(SF_ERR_INVALID, "NULL argument");
        if (bytes < 4096 || (bytes & (bytes - 1))) return fail(SF_ERR_INVALID, "bytes must be a power of two, at least 4096");
        if (reps == 0 || reps > 100000) return fail(SF_ERR_INVALID, "reps must be 1..100000");
        hipStream_t s = (hipStream_t)hip_stream;
        hipError_t he;
        unsigned g = grid;
        if (!g) {
            int dev = 0, cus = 0;
            if ((he = hipGetDevice(&dev)) != hipSuccess ||
                (he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
                return fail(SF_ERR_DEVICE, std::string("device query: ") + hipGetErrorString(he));
            g = (unsigned)std::max(cus, 1) * 32u - 1u;   // odd: see the header
        }
        float *sink = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto done = [&](int rc, const std::string &msg) {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (sink) (void)hipFree(sink);
            return rc ? fail(rc, msg) : ok();
        };
        if ((he = hipMalloc(&sink, 16)) != hipSuccess) return done(SF_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(he));
        if ((he = hipEventCreate(&e0)) != hipSuccess || (he = hipEventCreate(&e1)) != hipSuccess)
            return done(SF_ERR_DEVICE, std::string("event: ") + hipGetErrorString(he));
        // one untimed repetition first (fills the caches a resident buffer is read from)
        if ((he = sf::launch_read_probe(buf, bytes, 1, g, sink, s)) != hipSuccess ||
            (he = hipEventRecord(e0, s)) != hipSuccess ||
            (he = sf::launch_read_probe(buf, bytes, reps, g, sink, s)) != hipSuccess ||
            (he = hipEventRecord(e1, s)) != hipSuccess || (he = hipEventSynchronize(e1)) != hipSuccess)
            return done(SF_ERR_DEVICE, std::string("read probe: ") + hipGetErrorString(he));
        float ms = 0.f;
        if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
            return done(SF_ERR_DEVICE, std::string("event time: ") + hipGetErrorString(he));
        *ms_out = ms;
        return done(SF_OK, "");
    });
}

int verify_claim(sf_circuit_t *c, const double *claimed, uint64_t k, uint64_t index_seed, double f1,
                 uint64_t path_seed, double delta, uint32_t flags, void *hip_stream, void *workspace,
                 size_t workspace_bytes, double *f_e, int *passed)
{
    return guarded([&]() -> int {
        if (!c || !f_e || !passed || (k && !claimed)) return fail(SF_ERR_INVALID, "NULL argument");
        if (!c->has_cut) return fail(SF_ERR_NO_CUT, "set_cut has not been called");
        if (!(f1 > 0.0) || f1 > 1.0 || !(delta >= 0.0)) return fail(SF_ERR_INVALID, "bad f1 or delta");
        if (flags & ~uint32_t(SF_FP64_SWEEPS)) return fail(SF_ERR_INVALID, "unknown flag");
        if (k > (uint64_t(1) << 31)) return fail(SF_ERR_UNSUPPORTED, "more than 2^31 amplitudes");
        *f_e = 0.0;
        *passed = 0;
        if (!k) return fail(SF_ERR_INVALID, "no amplitudes");
        // step 1: the indices the Claimant was given; step 3: a fidelity-f1 simulation on them
        std::vector<uint64_t> idx(k);
        int rc = sample_bitstrings((uint32_t)c->n, k, index_seed, idx.data());
        if (rc) return rc;
        uint64_t m = 0;
        if ((rc = num_paths((uint32_t)c->k, f1, &m))) return rc;
        std::vector<uint64_t> ids(m);
        uint64_t got = 0;
        if ((rc = sample_paths((uint32_t)c->k, f1, path_seed, ids.data(), m, &got))) return rc;
        auto al = [](size_t x) { return (x + 255) / 256 * 256; };
        const size_t own = al(k * 8) + 2 * al(k * 16);
        char *base = nullptr;
        void *run_ws = nullptr;
        size_t run_ws_bytes = 0;
        bool allocated = false;
        hipError_t e;
        if (workspace) {
            if (workspace_bytes < own + (size_t(1) << 28)) return fail(SF_ERR_OOM, "workspace too small");
            base = (char *)workspace + (workspace_bytes - own) / 256 * 256;
            run_ws = workspace;
            run_ws_bytes = (size_t)(base - (char *)workspace);
        } else {
            if ((e = hipMalloc((void **)&base, own)) != hipSuccess) return fail(SF_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
            allocated = true;
        }
        hipStream_t s = (hipStream_t)hip_stream;
        auto finish = [&](int code) {
            if (allocated) { (void)hipStreamSynchronize(s); (void)hipFree(base); }
            return code;
        };
        uint64_t *d_bits = (uint64_t *)base;
        double *d_mine = (double *)(base + al(k * 8));
        double *d_claim = (double *)(base + al(k * 8) + al(k * 16));
        if ((e = hipMemcpyAsync(d_bits, idx.data(), k * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(d_claim, claimed, k * 16, hipMemcpyHostToDevice, s)) != hipSuccess)
            return finish(fail(SF_ERR_DEVICE, std::string("copy: ") + hipGetErrorString(e)));
        rc = run_paths(c, ids.data(), 0, got, d_bits, k, d_mine, flags | SF_BITS_ON_DEVICE | SF_OUT_ON_DEVICE,
                       hip_stream, run_ws, run_ws_bytes);
        if (rc) return finish(rc);
        // steps 5-6: estimate the fidelity between the two states and test it against f1
        double sm[4];
        if ((rc = overlap_sums(d_mine, d_claim, k, s, sm))) return finish(rc);
        *f_e = (sm[2] > 0.0 && sm[3] > 0.0) ? (sm[0] * sm[0] + sm[1] * sm[1]) / (sm[2] * sm[3]) : 0.0;
        *passed = std::fabs(*f_e - f1) <= delta ? 1 : 0;
        return finish(ok());
    });
}

}  // extern "C"
