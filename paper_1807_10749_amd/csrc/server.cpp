// Serving runtime: jobs (circuit, bitstrings, fidelity f) arrive at any time,
// are prepared (cut, path sample, memory estimate) on the server's own thread,
// admitted against a device-memory arena, and worked on in path chunks by a
// pool of workers, each with its own HIP stream.  A job that is admitted
// while others run starts at once on a free worker, so its kernels overlap
// with theirs on the device.  Which admitted job a free worker takes next is
// the server's policy: the oldest first (the default), round-robin, or the
// least remaining planned work first.  A job's FP64 partial sums stay
// resident in its arena slice until the last chunk; its result is then
// copied to host memory and its memory is released, which lets waiting jobs
// in.
//
// The memory a job asks for follows the per-process form of Section 9
// (M_proc = (C4 (2^q1 + 2^q2) + n_a) sizeof(complex)): block states for
// the tree levels of one chunk plus n_a bitstrings and accumulators.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sf_host.hpp"

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x) { return (x + 255) / 256 * 256; }

struct Job {
    uint64_t id = 0;
    sf_circuit_t *circ = nullptr;
    // request as submitted (prepared on the server's thread)
    uint64_t block_a_mask = 0;
    double f = 1.0;
    uint64_t path_seed = 0;
    double work = 0;                     // planned bytes of one chunk x chunks (policy SF_SERVE_LEAST_WORK)
    std::vector<uint64_t> bits;
    std::vector<uint64_t> paths;         // empty => all 2^k ids
    uint64_t n_paths = 0;
    uint32_t flags = 0;
    uint32_t k = 0;
    // memory
    size_t need = 0, ws_bytes = 0;
    size_t off = 0;                      // arena offset of [bits][acc][workspace]
    bool prepared = false, admitted = false, busy = false, done = false;
    int status = SF_OK;
    std::string error;
    uint64_t next_path = 0;              // index of the next path (range or list) to run
    uint64_t chunks_done = 0;
    std::vector<double> result;
    double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct sf_server {
    void *arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = false;
    uint64_t chunk_paths = 4096;
    std::map<size_t, size_t> free_list;  // offset -> size
    size_t in_use = 0, peak_in_use = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> preparing;      // submitted, not yet prepared (arrival order)
    std::deque<uint64_t> waiting;        // prepared, not admitted (arrival order)
    std::vector<uint64_t> active;        // admitted, not done
    size_t rr = 0;                       // round-robin cursor over active
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;
    std::thread prep_thread;
    uint32_t policy = SF_SERVE_OLDEST_FIRST;
    std::vector<hipStream_t> streams;
    double t0 = 0;
    uint64_t chunks_run = 0;
    int max_concurrent = 0, running = 0;

    bool alloc(size_t n, size_t &off)
    {
        for (auto it = free_list.begin(); it != free_list.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_list.erase(it);
                if (rest) free_list[off + n] = rest;
                in_use += n;
                peak_in_use = std::max(peak_in_use, in_use);
                return true;
            }
        }
        return false;
    }

    void release(size_t off, size_t n)
    {
        in_use -= n;
        auto it = free_list.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_list.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_list.erase(nx);
        }
        if (it != free_list.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_list.erase(it);
            }
        }
    }

    // admit waiting jobs that fit, in arrival order (a job that does not fit lets later,
    // smaller ones pass); caller holds mu
    void admit()
    {
        for (auto it = waiting.begin(); it != waiting.end();) {
            Job &j = *jobs[*it];
            size_t off = 0;
            if (j.need <= arena_bytes && alloc(j.need, off)) {
                j.off = off;
                j.admitted = true;
                j.t_admit = now_s() - t0;
                active.push_back(j.id);
                it = waiting.erase(it);
            } else {
                ++it;
            }
        }
    }

    // the next admitted job a free worker takes (one chunk per job at a time); caller holds mu
    Job *pick()
    {
        const size_t n = active.size();
        Job *best = nullptr;
        size_t best_i = 0;
        for (size_t i = 0; i < n; ++i) {
            const size_t at = policy == SF_SERVE_ROUND_ROBIN ? (rr + i) % n : i;
            Job &j = *jobs[active[at]];
            if (j.busy || j.done || j.next_path >= j.n_paths) continue;
            if (policy != SF_SERVE_LEAST_WORK) {      // active is in admission order
                best = &j;
                best_i = at;
                break;
            }
            const double left = j.work * (double)(j.n_paths - j.next_path) / (double)std::max<uint64_t>(j.n_paths, 1);
            const double bl = best ? best->work * (double)(best->n_paths - best->next_path) /
                                         (double)std::max<uint64_t>(best->n_paths, 1)
                                   : 0.0;
            if (!best || left < bl) { best = &j; best_i = at; }
        }
        if (best && policy == SF_SERVE_ROUND_ROBIN) rr = (best_i + 1) % std::max<size_t>(n, 1);
        return best;
    }

    // Host-side preparation of submitted jobs, off the callers' threads: cut, path sample,
    // memory estimate.  A job that fails here finishes with its error code.
    void prepare_loop()
    {
        for (;;) {
            Job *j = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [this] { return stop || !preparing.empty(); });
                if (preparing.empty()) return;
                j = jobs[preparing.front()].get();
            }
            std::string err;
            const int rc = prepare_job(*j, err);
            {
                std::lock_guard<std::mutex> lk(mu);
                preparing.pop_front();
                j->prepared = true;
                if (rc) {
                    j->status = rc;
                    j->error = err;
                    j->done = true;
                    j->t_done = now_s() - t0;
                    if (j->circ) { destroy_circuit(j->circ); j->circ = nullptr; }
                } else {
                    waiting.push_back(j->id);
                }
            }
            cv.notify_all();
        }
    }

    int prepare_job(Job &j, std::string &err)
    {
        uint64_t mask = j.block_a_mask;
        int rc;
        if (!mask && (rc = choose_cut(j.circ, &mask))) return (err = last_error(), rc);
        if ((rc = set_cut(j.circ, mask, &j.k))) return (err = last_error(), rc);
        if (j.f >= 1.0) {
            if (j.k > 40) return (err = "f = 1 with more than 2^40 paths", SF_ERR_UNSUPPORTED);
            j.n_paths = uint64_t(1) << j.k;
        } else {
            uint64_t m = 0;
            if ((rc = num_paths(j.k, j.f, &m))) return (err = last_error(), rc);
            j.paths.resize(m);
            if ((rc = sample_paths(j.k, j.f, j.path_seed, j.paths.data(), m, &m))) return (err = last_error(), rc);
            j.n_paths = m;
        }
        const int n = j.circ->n;
        const uint64_t all = n == 64 ? ~uint64_t(0) : ((uint64_t(1) << n) - 1);
        for (uint64_t b : j.bits)
            if (b & ~all) return (err = "bitstring has bits outside the grid", SF_ERR_INVALID);
        const uint64_t chunk = std::min<uint64_t>(chunk_paths, j.n_paths);
        size_t est = 0;
        workspace_size(j.circ, chunk, j.bits.size(), j.flags, &est);
        // at least 256 MiB (run_paths' minimum), at most a quarter of the arena: run_paths
        // processes the tree in smaller batches when its workspace is below the estimate
        j.ws_bytes = std::max<size_t>(size_t(1) << 28, std::min(est, arena_bytes / 4));
        j.need = align_up(j.bits.size() * 8) + align_up(j.bits.size() * 16) + align_up(j.ws_bytes);
        if (j.need > arena_bytes) return (err = "job larger than the arena", SF_ERR_OOM);
        // planned work of the first chunk (sweep and gather bytes, no device work) times the
        // number of chunks: the remaining-work key of SF_SERVE_LEAST_WORK
        if (policy == SF_SERVE_LEAST_WORK && chunk) {
            std::string e2;
            const uint32_t fl = j.flags | SF_OUT_ON_DEVICE;
            if (sf::execute(*j.circ, j.paths.empty() ? nullptr : j.paths.data(), 0, chunk, j.bits.data(),
                            j.bits.size(), nullptr, fl, nullptr, nullptr, 0, e2, true) == SF_OK) {
                const sf_run_stats_t &st = j.circ->stats;
                j.work = (double)(st.sweep_bytes + st.gather_bytes) * (double)((j.n_paths + chunk - 1) / chunk);
            }
        }
        return SF_OK;
    }

    void worker(int w)
    {
        hipStream_t s = streams[w];
        for (;;) {
            Job *j = nullptr;
            uint64_t first = 0, count = 0;
            {
                std::unique_lock<std::mutex> lk(mu);
                for (;;) {
                    admit();
                    j = pick();
                    if (j || stop) break;
                    cv.wait(lk);
                }
                if (!j) return;
                j->busy = true;
                first = j->next_path;
                count = std::min<uint64_t>(chunk_paths, j->n_paths - first);
                j->next_path += count;
                ++running;
                max_concurrent = std::max(max_concurrent, running);
            }
            char *base = (char *)arena + j->off;
            const size_t nb = j->bits.size();
            uint64_t *d_bits = (uint64_t *)base;
            double *d_acc = (double *)(base + align_up(nb * 8));
            char *ws = base + align_up(nb * 8) + align_up(nb * 16);
            int rc = SF_OK;
            std::string err;
            if (first == 0 && nb) {
                hipError_t he = hipMemcpyAsync(d_bits, j->bits.data(), nb * 8, hipMemcpyHostToDevice, s);
                if (he != hipSuccess) { rc = SF_ERR_DEVICE; err = hipGetErrorString(he); }
            }
            if (rc == SF_OK) {
                const uint32_t fl = j->flags | SF_OUT_ON_DEVICE | SF_BITS_ON_DEVICE | (first ? SF_ACCUMULATE : 0u);
                const uint64_t *ids = j->paths.empty() ? nullptr : j->paths.data() + first;
                rc = run_paths(j->circ, ids, j->paths.empty() ? first : 0, count, d_bits, nb, d_acc, fl, s, ws,
                               j->ws_bytes);
                if (rc) err = last_error();
            }
            bool finished = false;
            if (rc == SF_OK && first + count == j->n_paths) {
                j->result.resize(2 * nb);
                hipError_t he = hipMemcpyAsync(j->result.data(), d_acc, nb * 16, hipMemcpyDeviceToHost, s);
                if (he == hipSuccess) he = hipStreamSynchronize(s);
                if (he != hipSuccess) { rc = SF_ERR_DEVICE; err = hipGetErrorString(he); }
                finished = true;
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                --running;
                ++chunks_run;
                j->busy = false;
                j->chunks_done++;
                if (rc != SF_OK) { j->status = rc; j->error = err; finished = true; }
                if (finished) {
                    j->done = true;
                    j->t_done = now_s() - t0;
                    release(j->off, j->need);
                    active.erase(std::find(active.begin(), active.end(), j->id));
                    destroy_circuit(j->circ);
                    j->circ = nullptr;
                }
            }
            cv.notify_all();
        }
    }
};

namespace {
thread_local std::string g_srv_err;
int sfail(int code, const std::string &m) { g_srv_err = m; return code; }
}  // namespace

extern "C" {

const char *server_last_error(void) { return g_srv_err.c_str(); }

int server_create(size_t arena_bytes, void *arena, uint32_t n_workers, uint64_t chunk_paths, sf_server_t **out)
{
    try {
        if (!out) return sfail(SF_ERR_INVALID, "out is NULL");
        *out = nullptr;
        if (n_workers < 1 || n_workers > 16) return sfail(SF_ERR_INVALID, "1..16 workers");
        if (arena_bytes < (size_t(1) << 28)) return sfail(SF_ERR_INVALID, "arena smaller than 256 MiB");
        auto *s = new sf_server();
        s->arena_bytes = arena_bytes;
        s->chunk_paths = chunk_paths ? chunk_paths : 4096;
        if (arena) {
            s->arena = arena;
        } else {
            hipError_t he = hipMalloc(&s->arena, arena_bytes);
            if (he != hipSuccess) { delete s; return sfail(SF_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(he)); }
            s->own_arena = true;
        }
        s->free_list[0] = arena_bytes;
        s->t0 = now_s();
        for (uint32_t w = 0; w < n_workers; ++w) {
            hipStream_t st;
            hipError_t he = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (he != hipSuccess) {
                for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
                if (s->own_arena) (void)hipFree(s->arena);
                delete s;
                return sfail(SF_ERR_DEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(he));
            }
            s->streams.push_back(st);
        }
        for (uint32_t w = 0; w < n_workers; ++w) s->workers.emplace_back([s, w] { s->worker((int)w); });
        s->prep_thread = std::thread([s] { s->prepare_loop(); });
        *out = s;
        return SF_OK;
    } catch (const std::exception &e) {
        return sfail(SF_ERR_INVALID, e.what());
    }
}

int server_submit(sf_server_t *s, const sf_job_t *job, uint64_t *job_id)
{
    try {
        const double t_entry = s ? now_s() - s->t0 : 0.0;
        if (!s || !job || !job_id) return sfail(SF_ERR_INVALID, "NULL argument");
        if (job->n_bits && !job->bitstrings) return sfail(SF_ERR_INVALID, "bitstrings is NULL");
        if (job->flags & ~uint32_t(SF_FP64_SWEEPS)) return sfail(SF_ERR_INVALID, "only SF_FP64_SWEEPS may be set");
        if (job->n_bits > (size_t)INT_MAX) return sfail(SF_ERR_UNSUPPORTED, "more than 2^31 - 1 bitstrings");
        // the smallest arena slice a job can have: its bitstrings, FP64 sums and a 256 MiB workspace
        if (align_up(job->n_bits * 8) + align_up(job->n_bits * 16) + (size_t(1) << 28) > s->arena_bytes)
            return sfail(SF_ERR_OOM, "job larger than the arena");
        auto j = std::make_unique<Job>();
        int rc = create_circuit(job->rows, job->cols, job->gates, job->n_gates, &j->circ);
        if (rc) return sfail(rc, last_error());
        j->block_a_mask = job->block_a_mask;
        j->f = job->f;
        j->path_seed = job->path_seed;
        j->flags = job->flags;
        j->bits.assign(job->bitstrings, job->bitstrings + job->n_bits);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            j->id = s->next_id++;
            j->t_submit = t_entry;
            *job_id = j->id;
            s->preparing.push_back(j->id);
            s->jobs[j->id] = std::move(j);
        }
        s->cv.notify_all();
        return SF_OK;
    } catch (const std::exception &e) {
        return sfail(SF_ERR_INVALID, e.what());
    }
}

int server_set_policy(sf_server_t *s, uint32_t policy)
{
    if (!s) return sfail(SF_ERR_INVALID, "server is NULL");
    if (policy > SF_SERVE_LEAST_WORK) return sfail(SF_ERR_INVALID, "unknown policy");
    std::lock_guard<std::mutex> lk(s->mu);
    s->policy = policy;
    return SF_OK;
}

int server_poll(sf_server_t *s, uint64_t job_id, double *amps, sf_job_info_t *info)
{
    if (!s) return sfail(SF_ERR_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return sfail(SF_ERR_INVALID, "unknown job");
    Job &j = *it->second;
    if (info) {
        info->t_submit = j.t_submit;
        info->t_admit = j.t_admit;
        info->t_done = j.t_done;
        info->n_paths = j.prepared ? j.n_paths : 0;
        info->k = j.prepared ? j.k : 0;
        info->chunks = (uint32_t)j.chunks_done;
        info->status = j.done ? j.status : SF_PENDING;
    }
    if (!j.done) return SF_PENDING;
    if (j.status != SF_OK) return sfail(j.status, j.error);
    if (amps && !j.result.empty()) std::memcpy(amps, j.result.data(), j.result.size() * sizeof(double));
    return SF_OK;
}

int server_release(sf_server_t *s, uint64_t job_id)
{
    if (!s) return sfail(SF_ERR_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return sfail(SF_ERR_INVALID, "unknown job");
    if (!it->second->done) return sfail(SF_ERR_INVALID, "job not finished");
    s->jobs.erase(it);
    return SF_OK;
}

int server_drain(sf_server_t *s)
{
    if (!s) return sfail(SF_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [s] { return s->preparing.empty() && s->waiting.empty() && s->active.empty(); });
    return SF_OK;
}

int server_stats(sf_server_t *s, sf_server_stats_t *out)
{
    if (!s || !out) return sfail(SF_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->arena_bytes = s->arena_bytes;
    out->peak_bytes = s->peak_in_use;
    out->in_use_bytes = s->in_use;
    out->chunks = s->chunks_run;
    out->max_concurrent_chunks = (uint32_t)s->max_concurrent;
    out->waiting = (uint32_t)(s->waiting.size() + s->preparing.size());
    out->active = (uint32_t)s->active.size();
    return SF_OK;
}

int server_destroy(sf_server_t *s)
{
    if (!s) return SF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (std::thread &t : s->workers) t.join();
    if (s->prep_thread.joinable()) s->prep_thread.join();
    for (auto &kv : s->jobs)
        if (kv.second->circ) destroy_circuit(kv.second->circ);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->own_arena) (void)hipFree(s->arena);
    delete s;
    return SF_OK;
}

}  // extern "C"
