/*
 * sfpath.h -- C ABI of the MI355X Schroedinger-Feynman path-sum library.
 *
 * Method (arXiv:1807.10749): the qubit grid is cut into block A (which
 * holds qubit 0) and block B (Section 2; Section 9, "Performance
 * estimation": a single straight-line cut).  Every CZ that crosses the cut
 * is split as P0 (x) I + P1 (x) Z (Section 2, Eq. (CZ)) and every crossing
 * iSWAP into the four terms of Eq. (4way), so crossing gates deciding k path
 * bits give 2^k paths and |psi> = sum_j |phi_j> (Section 3).  Each path evolves
 * the two blocks separately; requested amplitudes are accumulated over paths
 * as amp(x) = sum_p psiA_p(x_A) psiB_p(x_B) (Section 2, "Final-state
 * amplitudes").  Summing a fraction f of the paths trades fidelity for time
 * (Section 3, Eq. (fid)).
 *
 * Conventions:
 *   - qubit id on an R x C grid is r*C + c; bitstring bit q = value of qubit
 *     q (x is a uint64); x_A / x_B are the bits of x at the block's qubits,
 *     packed in ascending qubit order;
 *   - gate kinds 0 H, 1 X^1/2, 2 Y^1/2, 3 T, 4 CZ, 5 iSWAP with
 *     H = [[1,1],[1,-1]]/sqrt2, X^1/2 = [[1+i,1-i],[1-i,1+i]]/2,
 *     Y^1/2 = [[1+i,-1-i],[1+i,1+i]]/2, T = diag(1, e^{i pi/4}),
 *     iSWAP: |01> -> i|10>, |10> -> i|01>, |00> and |11> kept (Section 7);
 *   - the crossing gates are ordered by (cycle, smaller qubit id); a crossing
 *     CZ takes one path bit, a crossing iSWAP two, and the earliest gate the
 *     most significant bits (so an aligned block of 2^b ids shares its
 *     prefix).  CZ bit 0 takes P0 on the A endpoint, bit 1 takes P1 on the A
 *     endpoint and Z on the B endpoint.  iSWAP bits r = 2i + j take the term
 *     |i><j| (x) G_ij of Eq. (4way), |i><j| on the A endpoint and the 2x2 block
 *     G_ij (rows 2i.., columns 2j.. of the matrix in the basis 2 x_A + x_B) on
 *     the B endpoint.
 *
 * Errors: every function returns 0 on success or a negative code below and
 * never throws; last_error() gives a message for the calling thread.
 * Device errors of asynchronous work surface at the next synchronising call.
 */
#ifndef SFPATH_H
#define SFPATH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SF_OK              0
#define SF_ERR_INVALID   (-1)  /* bad argument: qubit outside the grid, non-adjacent two-qubit gate, id >= 2^k ... */
#define SF_ERR_OOM       (-2)  /* host or device memory, or a workspace that is too small */
#define SF_ERR_UNSUPPORTED (-3) /* n > 64, a block > 30 qubits, k > 62, ... */
#define SF_ERR_NO_CUT    (-4)  /* run_paths before set_cut */
#define SF_ERR_DEVICE    (-5)  /* HIP runtime error (no GPU, launch failure, fault) */

/* One gate record, 8 bytes. q1 is ignored for one-qubit gates. */
typedef struct {
    uint8_t kind;     /* 0 H, 1 X^1/2, 2 Y^1/2, 3 T, 4 CZ, 5 iSWAP */
    uint8_t pad;
    uint16_t cycle;   /* clock cycle; must not decrease along the list */
    uint16_t q0, q1;
} sf_gate_t;

typedef struct sf_circuit sf_circuit_t;   /* opaque, library-owned */

/* run_paths flags */
#define SF_ACCUMULATE     1u   /* add into amps instead of overwriting */
#define SF_OUT_ON_DEVICE  2u   /* amps is a device pointer */
#define SF_FP64_SWEEPS    4u   /* evolve the blocks in complex128 instead of complex64 */
#define SF_PLAIN          8u   /* one path at a time, no batching, no shared prefixes */
#define SF_BITS_ON_DEVICE 16u  /* bitstrings is a device pointer */
#define SF_TIMING         32u  /* time every kernel with HIP events (see get_run_stats) */

/* rejection-sampling flag (rejection_m, rejection_accept, frugal_sample) */
#define SF_SAMPLE_BASIC   256u /* Algorithm 1 instead of Algorithm 2 */

/*
 * create_circuit: copy a gate list on an R x C grid (rows*cols <= 64).
 * Gates must act on grid qubits; a CZ or iSWAP must join grid neighbours; cycles
 * must not decrease along the list and a qubit may appear at most once per
 * cycle (Section 1 circuits: one layer of gates per clock cycle).
 * The library owns *out until destroy_circuit.
 */
int create_circuit(int rows, int cols, const sf_gate_t *gates, size_t n_gates,
                   sf_circuit_t **out);

/* destroy_circuit: free the circuit, its plans and any device memory it holds. */
int destroy_circuit(sf_circuit_t *c);

/*
 * set_cut: choose block A as the qubits whose bits are set in block_a_mask
 * (bit 0 must be set; block B is the rest of the grid and must not be empty;
 * each block at most 30 qubits).  Writes the number k of path bits of the
 * crossing gates (Section 2: "cross-block" CZ gates, xCZ, one bit each; a
 * crossing iSWAP two, Section 7) to *k_out.  Plans are rebuilt.
 */
int set_cut(sf_circuit_t *c, uint64_t block_a_mask, uint32_t *k_out);

/*
 * choose_cut: the straight-line cut of Section 9 (Performance estimation):
 * among all vertical and horizontal grid cuts, minimise the larger block,
 * then the path bits of the crossing gates; ties prefer vertical cuts, then the cut
 * nearest to column/row 0.  Writes block A's mask (holding qubit 0).
 */
int choose_cut(const sf_circuit_t *c, uint64_t *block_a_mask);

/*
 * num_paths: ceil(f * 2^k), the number of paths kept at fidelity f
 * (Section 3, Eq. (fid)); 0 < f <= 1, k <= 62.
 */
int num_paths(uint32_t k, double f, uint64_t *n_out);

/*
 * sample_paths: ceil(f * 2^k) distinct path ids, uniform, sorted ascending
 * (Section 3: which terms are kept does not matter for these circuits).
 * Floyd's algorithm (Bentley & Floyd 1987) over SplitMix64 (Steele, Lea &
 * Flood 2014) seeded with `seed`; a bounded draw in [0, m) is
 * floor(r * m / 2^64) for a 64-bit output r.  `out` is host memory with
 * room for `cap` ids.
 */
int sample_paths(uint32_t k, double f, uint64_t seed, uint64_t *out, uint64_t cap,
                 uint64_t *n_out);

/*
 * run_paths: amps[j] = sum over the given paths p of psiA_p(x_A) psiB_p(x_B)
 * for x = bitstrings[j] (plus the previous content of amps with
 * SF_ACCUMULATE).  The raw partial sum is returned: no 1/sqrt(f) rescale.
 *   path_ids   host array of n_paths distinct ids < 2^k, or NULL for the
 *              range [path_begin, path_begin + n_paths);
 *   bitstrings n_bits uint64 values < 2^n (host, or device with
 *              SF_BITS_ON_DEVICE); n_bits <= 2^31 - 1, else
 *              SF_ERR_UNSUPPORTED;
 *   amps       2*n_bits doubles (re, im), host or device (SF_OUT_ON_DEVICE);
 *   hip_stream hipStream_t to enqueue on (NULL = default stream);
 *   workspace  caller-owned device memory of workspace_bytes, or NULL to let
 *              the library allocate (and keep, until destroy_circuit) what
 *              it needs.  A non-NULL workspace smaller than 256 MiB or than
 *              one slot per tree level is rejected with SF_ERR_OOM.
 * Returns after the work has finished (the stream is synchronised).
 * Blocks evolve in complex64 (complex128 with SF_FP64_SWEEPS); the
 * cross-path sum is formed in FP64.
 * Paths whose term is exactly zero are skipped: a qubit that receives two
 * cut-gate projectors with only diagonal gates on it in between keeps a
 * nonzero amplitude only if both path bits agree (Section 2: the projectors
 * of Eq. (CZ) leave zero blocks, which the simulator skips; here whole zero
 * states).  get_run_stats reports how many requested paths remained.
 */
int run_paths(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin,
              uint64_t n_paths, const uint64_t *bitstrings, size_t n_bits,
              double *amps, uint32_t flags, void *hip_stream,
              void *workspace, size_t workspace_bytes);

/*
 * run_paths_noalloc: run_paths for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * results as run_paths with SF_BITS_ON_DEVICE | SF_OUT_ON_DEVICE (both required; SF_TIMING is
 * refused), but the workspace is a fixed 64 MiB device array of the library, one per GPU, held
 * until the process ends; the call makes no device allocation.  A request whose workspace does
 * not fit in 64 MiB (bitstring indices and visiting order, slot tables, pass programs, one
 * block-state slot per tree level) returns SF_ERR_OOM with that reason.  Every call on a GPU
 * uses that GPU's one array: calls that overlap on one GPU (other threads or streams) race and
 * must be serialised by the caller; each call initialises what it reads.  With tuning jit it
 * compiles nothing (loading a compiled kernel allocates device memory for its code): passes
 * whose kernel an earlier call of the process compiled run it, the others run interpreted.
 */
int run_paths_noalloc(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin,
                      uint64_t n_paths, const uint64_t *bitstrings, size_t n_bits,
                      double *amps, uint32_t flags, void *hip_stream);

/*
 * workspace_size: device bytes run_paths would use for a request of
 * n_paths paths and n_bits bitstrings with the current tuning when it
 * may keep every tree level of the request resident (the library then
 * runs the levels breadth-first).  Any workspace of at least 256 MiB
 * works; smaller ones make run_paths process the tree in more batches.
 */
int workspace_size(const sf_circuit_t *c, uint64_t n_paths, size_t n_bits, uint32_t flags,
                   size_t *bytes);

/* Tuning knobs (see set_tuning / autotune). 0 = library default. */
typedef struct {
    uint32_t reg_qubits;     /* qubits held in registers per pass, 1..5 (1..4 with SF_FP64_SWEEPS) */
    uint32_t leaf_batch;     /* max paths per leaf batch (power of two) */
    uint32_t max_slots;      /* max slots of any batch (power of two) */
    uint32_t waves_per_cu;   /* grid cap of the sweep kernels in waves per compute unit
                                (default 128; 4 waves per workgroup) */
    uint32_t dense_qubits;   /* 0: gates on registers and lanes only; 2..4: also fuse windows of up to
                                this many qubits into dense 16 x 16 blocks applied on matrix cores
                                (complex64 sweeps only) */
    uint32_t no_leaf_fold;   /* 0: when every non-diagonal gate of the last tree level(s) acts
                                on a branch qubit of those levels, the gather reads the level
                                above and applies them itself (their states are never written);
                                1: always write the leaf states and gather from them */
    uint32_t fold_levels;    /* most trailing tree levels folded into the gather (0: as many as
                                qualify, up to 5 path bits; a group of levels qualifies when all
                                its non-diagonal gates act on its branch qubits) */
    uint32_t chain_passes;   /* 0: one launch per pass; 1: consecutive small passes of one kernel
                                variant (each at most one workgroup per compute unit) run as one
                                persistent cooperative launch with a grid barrier between them.
                                The barrier costs more than a kernel boundary between back-to-back
                                launches on one stream, so 0 is the default */
    uint32_t no_row_skip;    /* 0: the last pass of each block at the level the path sum reads
                                computes only the tiles holding rows the requested bitstrings
                                read (when they are expected to be under 80% of its tiles);
                                1: whole states */
    uint32_t no_defer;       /* 0: when block A's part of the level the general fold reads is only
                                its crossing gates' projectors and one-qubit gates on the projected
                                qubits, that level's block-A states are not written: the fold
                                reads the level above with the projected bits set and applies
                                the gates itself; 1: always write them */
    uint32_t no_chain_merge; /* 0: a run of consecutive chain levels (every node one child) is
                                planned as one segment, its operations sharing passes, when that
                                takes no more passes than planning the levels one by one (the
                                root joins the run below it); 1: one segment per level */
    uint32_t jit;            /* 0: the pass kernels interpret each pass program (read per tile from
                                LDS); 1: every pass outside a chained launch that is not a dense
                                block runs a kernel compiled at run time for its program (hiprtc,
                                a few seconds per distinct set of programs, cached for the
                                process): the gates' kinds and positions become constants, which
                                removes the interpreter's per-operation register copies and
                                selects.  Results agree with the interpreted passes to rounding */
    uint32_t no_tail_move;   /* 0: a block whose segment ends in an in-place pass and whose
                                children are written by a fan-out (at most 16 children per parent)
                                leaves that last pass to the children's first pass when their plan
                                takes no more passes with it: one read and write of the parent
                                batch saved, that pass's gates run once per child; 1: never */
} sf_tuning_t;

int set_tuning(sf_circuit_t *c, const sf_tuning_t *t);
int get_tuning(const sf_circuit_t *c, sf_tuning_t *t);

/*
 * autotune: choose the tuning for requests shaped like this one.  Every
 * candidate (register qubits per pass x leaf-batch size x grid size per
 * compute unit) is first planned without device work and ranked by a cost
 * model of the form of Section 9, Eq. (t_tot): the planned sweep bytes and
 * gather bytes over measured bandwidths plus a per-launch cost (the paper's
 * C1 2^x_p (q1 2^q1 + q2 2^q2)(d_p + C2 2^x_b d_b) + C3 2^(x_p+x_b) n_a
 * with the constants taken from the device).  The best-ranked candidate of
 * every kind (folded levels or written leaves; no dense blocks, or dense
 * windows of up to 2, 3 or 4 qubits), more
 * candidates by rank up to n_measure, and the current tuning are then timed
 * with real run_paths
 * calls on this request (same argument rules as run_paths, checked before
 * any device work; amps is overwritten, so SF_ACCUMULATE is rejected with
 * SF_ERR_INVALID) and the fastest is kept on the circuit and written to *best.
 * Results are cached for the process per (device kind, block sizes, k, tree
 * levels, number of paths, number of bitstrings, flags); see
 * save_tuning_cache / load_tuning_cache to keep them across processes.
 */
int autotune(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
             const uint64_t *bitstrings, size_t n_bits, double *amps, uint32_t flags,
             void *hip_stream, void *workspace, size_t workspace_bytes, uint32_t n_measure,
             sf_tuning_t *best);

/*
 * save_tuning_cache: write every tuning autotune has chosen in this process
 * (or loaded) to the text file at path, one entry per line:
 *   <device arch>:<compute units>/<qA>/<qB>/<k>/<levels>/<paths>/<bitstrings>/<flags>
 *   reg_qubits leaf_batch max_slots waves_per_cu dense_qubits no_leaf_fold fold_levels
 * (lines starting with '#' are comments).  The file is overwritten.
 * SF_ERR_INVALID if path is NULL or cannot be written.
 *
 * load_tuning_cache: add the entries of such a file to the process cache
 * (an entry with the same key replaces the cached one); a later autotune of a
 * request with that key on that kind of device takes the stored tuning
 * without measuring.  Writes the number of entries read to *n_loaded (may be
 * NULL).  SF_ERR_INVALID if the file cannot be read or a line is malformed or
 * out of range (then nothing is added).  Both are thread-safe.
 */
int save_tuning_cache(const char *path);
int load_tuning_cache(const char *path, uint32_t *n_loaded);

/* Statistics of the last run_paths call on this circuit. Times are only
 * filled when the run used SF_TIMING. */
typedef struct {
    double ms_total;         /* host wall time of run_paths */
    double ms_sweep;         /* summed kernel time of gate-sweep passes */
    double ms_gather;        /* summed kernel time of gather / path-sum */
    double ms_other;         /* init, pext, zero fill */
    uint64_t n_sweep_launches;
    uint64_t n_gather_launches;
    uint64_t sweep_bytes;    /* algorithmic bytes of the sweep passes: each writes the slots in
                                use of its state once and reads its source once (a fan-out: the
                                parent slots of its children; amplitudes in a known zero
                                subspace excluded) */
    uint64_t gather_bytes;   /* algorithmic bytes of gather launches in their visiting order:
                                block-A rows once per group of bitstrings that read the same
                                block-A rows, block-B rows once per bitstring, plus indices
                                and the amplitudes read and written */
    uint64_t n_batches;      /* leaf batches */
    uint64_t n_passes_a, n_passes_b;  /* passes per leaf path of block A / B (full plan) */
    uint64_t gather_row_bytes;  /* rows of both blocks read once per bitstring (no reuse) */
    uint64_t a_groups;       /* groups of bitstrings that share their block-A rows (estimated
                                from the bitstring count in a planning-only run) */
    double ms_plan;          /* host time from entry to the first enqueued device operation */
    uint64_t n_paths_live;   /* requested paths whose term is not known to be zero (see run_paths) */
    uint64_t n_chained_passes;  /* sweep passes run inside chained launches (see chain_passes); a chain
                                   counts once in n_sweep_launches */
    uint64_t gather_ws_bytes;   /* largest block-B state one gather launch reads rows of (slots x 2^qB x
                                   element size): every bitstring reads rows anywhere in it, so this working
                                   set decides which level of the memory hierarchy serves the path sum */
    double row_mask_frac[2];    /* per block: fraction of the tiles of its last pass before the path sum
                                   that were computed (the rest hold no row a requested bitstring reads;
                                   tuning no_row_skip); 0 when that pass computed every tile */
    uint64_t n_jit_passes;      /* sweep passes run by kernels compiled for their program (tuning jit) */
    double jit_compile_ms;      /* host time this call spent compiling such kernels (0 when all were
                                   compiled by earlier calls of the process) */
} sf_run_stats_t;

int get_run_stats(const sf_circuit_t *c, sf_run_stats_t *s);

/*
 * describe_plan: human-readable summary of the block programs: per tree level
 * and block the number of operations and of fused passes, planned for the
 * slot count an all-paths run uses at that level (2^bits, capped by the
 * tuning).  Each pass reads "<non-diagonal gates>g/<diagonal groups>d" (or
 * "dense"), with "/z<N>" when its source state has a known zero subspace on N
 * projected qubits (Section 2 zero blocks: a crossing gate's projector not yet
 * followed by a non-diagonal gate on its qubit).  Host only, no device work.
 * Writes a NUL-terminated string of at most cap bytes.
 */
int describe_plan(sf_circuit_t *c, char *out, size_t cap);

/*
 * compile_segment_kernels: the kernels that tuning jit = 1 compiles for the passes of one block
 * (half 0 = A, 1 = B) over tree levels first_level..last_level planned as one segment for 2^slot_bits
 * slots and reg_qubits register qubits (complex128 states when fp64 is nonzero, reg_qubits <= 4),
 * one kernel per pass that is not a dense block, compiled for gfx950 with hiprtc on the host and
 * discarded (no device is needed or used).  *n_kernels (host) receives their number and
 * *code_bytes (host) the total code-object size.  For checking the generated kernels on a
 * machine without a GPU.  SF_ERR_INVALID on NULL pointers or out-of-range arguments,
 * SF_ERR_NO_CUT before set_cut, SF_ERR_UNSUPPORTED if the segment cannot be planned or a kernel
 * does not compile (the compiler's log in last_error).
 */
int compile_segment_kernels(sf_circuit_t *c, int half, uint32_t first_level, uint32_t last_level,
                            uint32_t slot_bits, uint32_t reg_qubits, uint32_t fp64, uint32_t *n_kernels,
                            uint64_t *code_bytes);

/* Message for the last error on the calling thread ("" if none). */
const char *last_error(void);

/*
 * Rejection sampling of bitstrings from a batch of output probabilities
 * (Section "Frugal rejection sampling" and its figure: Algorithm 1, basic;
 * Algorithm 2, frugal).  N = 2^n for n qubits.
 *
 * rejection_m: step 1.  Algorithm 2 (flags 0): the smallest integer M' >= 1
 * with e^{-M'} (1 + M') <= eps, the probability mass above M'/N under
 * Porter-Thomas statistics (M' = 10 for eps = 5e-4).  Algorithm 1
 * (SF_SAMPLE_BASIC): M = ceil(ln(N / eps)) (41 for eps = 1e-3, n = 49).
 * Host only; SF_ERR_INVALID for n outside 1..64 or eps outside (0, 1).
 */
int rejection_m(uint32_t n_qubits, double eps, uint32_t flags, double *m);

/*
 * sample_bitstrings: step 2.  count distinct uniform n-qubit bitstrings into
 * the host array out (bit q = qubit q): draw i is output i of
 * SplitMix64(seed) masked to n bits, repeats are skipped, the kept draws stay
 * in draw order.  SF_ERR_INVALID if count exceeds 2^n.
 */
int sample_bitstrings(uint32_t n_qubits, uint64_t count, uint64_t seed, uint64_t *out);

/* rejection_workspace_size: device bytes rejection_accept needs for n candidates. */
int rejection_workspace_size(uint64_t n, size_t *bytes);

/*
 * rejection_accept: step 4 of Algorithm 2 (steps 4-5 of Algorithm 1 with
 * SF_SAMPLE_BASIC) on the device.  amps: n FP64 complex amplitudes (re, im
 * interleaved, device, as run_paths writes them with SF_OUT_ON_DEVICE) of
 * candidates drawn uniformly.  For candidate j: p = re^2 + im^2, t = p N / M,
 * u = (output j of SplitMix64(seed) >> 11) * 2^-53, every product and sum
 * rounded on its own in FP64; Algorithm 2 accepts when u < t, i.e. with
 * probability min{1, p N / M'}; Algorithm 1 removes candidates with t > 1
 * (p > M/N) and accepts the others when u < t.  accepted (device, capacity
 * n) receives the indices of the accepted candidates in ascending order,
 * *n_accepted (host) their number, *err_est (host) the batch estimate
 * (N / n) sum_{t > 1} p of the probability mass above M/N (the sampling error
 * the paper computes per batch when Porter-Thomas statistics are not
 * assumed).  workspace: device scratch of rejection_workspace_size(n) bytes,
 * owned by the caller.  Synchronizes hip_stream before returning.
 */
int rejection_accept(const double *amps, uint64_t n, uint32_t n_qubits, double m, uint64_t seed,
                     uint32_t flags, uint32_t *accepted, uint64_t *n_accepted, double *err_est,
                     void *hip_stream, void *workspace, size_t workspace_bytes);

/*
 * frugal_sample: Algorithm 2 (Algorithm 1 with SF_SAMPLE_BASIC) end to end:
 * n_candidates candidates from sample_bitstrings(seed_candidates), their
 * amplitudes by run_paths over the given paths (path_ids / path_begin /
 * n_paths as in run_paths; flags may add SF_FP64_SWEEPS or SF_PLAIN), and
 * rejection_accept with m and seed_accept.  The accepted bitstrings go to the
 * host array out (capacity n_candidates) in candidate order, their number to
 * *n_out, the batch's error estimate to *err_est.  With a caller workspace,
 * 28 B per candidate plus the acceptance scratch are taken from its end and
 * run_paths gets the rest (at least 256 MiB must remain); without one the
 * library allocates.  The probability of a path-sum subset is |amp|^2 of the
 * partial sum (Section 3: the sum over a fraction f of the paths).
 */
int frugal_sample(sf_circuit_t *c, const uint64_t *path_ids, uint64_t path_begin, uint64_t n_paths,
                  uint64_t n_candidates, double m, uint64_t seed_candidates, uint64_t seed_accept,
                  uint32_t flags, void *hip_stream, void *workspace, size_t workspace_bytes,
                  uint64_t *out, uint64_t *n_out, double *err_est);

/*
 * Validation of results (appendix on validating simulation results).
 *
 * fidelity_estimate: the state overlap estimated from n amplitudes of two
 * states at the same indices (device arrays, FP64 complex, re/im
 * interleaved): f_e = |sum conj(a) b|^2 / (sum |a|^2 sum |b|^2); the sums
 * are FP64, per block in a fixed order, then over blocks in block order on
 * the host.  Optionally returns sum |a|^2 and sum |b|^2 (norm_a, norm_b may
 * be NULL).  Synchronizes hip_stream.
 */
int fidelity_estimate(const double *a, const double *b, uint64_t n, void *hip_stream, double *f_e,
                      double *norm_a, double *norm_b);

/*
 * xeb_fidelity: linear cross-entropy fidelity N <|a|^2> - 1 of n sampled
 * bitstrings' ideal amplitudes (device, FP64 complex), N = 2^n_qubits (the
 * cross-entropy check the paper mentions beside the overlap estimate).
 */
int xeb_fidelity(const double *amps, uint64_t n, uint32_t n_qubits, void *hip_stream, double *f);

/*
 * read_bandwidth: measured read ceiling of one level of the memory hierarchy,
 * for the rooflines of the path-sum kernels, whose working sets live in the
 * caches rather than in HBM.  Reads the first `bytes` (a power of two, at
 * least 4096) of the device buffer `buf` `reps` times in one launch of a
 * streaming kernel with eight 16-byte loads in flight per thread: a buffer
 * far larger than the Infinity Cache measures HBM, one that fits the
 * Infinity Cache but not an XCD's L2 (4 MB) measures the Infinity Cache, one
 * that fits an XCD's L2 measures L2.
 * `grid` workgroups of 256 threads (0: 32 per compute unit less one; with an
 * odd count every workgroup's reads walk the whole buffer instead of
 * revisiting a few 4 KB chunks that its XCD's L2 would keep).  Enqueued on
 * hip_stream, which the call synchronizes; ms_out = launch time from events
 * on that stream.  The buffer is only read; its contents do not matter.
 */
int read_bandwidth(const void *buf, size_t bytes, uint32_t reps, uint32_t grid, void *hip_stream, double *ms_out);

/*
 * verify_claim: the Verifier's side of the two-party validation protocol.
 * Step 1: the k indices are sample_bitstrings(n, k, index_seed); the
 * Claimant's amplitudes at them (claimed, host, k FP64 complex) are the
 * input.  Step 3: the Verifier simulates with fidelity f1 (the paths
 * sample_paths(k_cut, f1, path_seed), run_paths on the k indices).  Steps 5-6:
 * *f_e = fidelity_estimate(Verifier's, Claimant's amplitudes) and *passed =
 * |f_e - f1| <= delta.  flags may be SF_FP64_SWEEPS.  The workspace is used
 * as in frugal_sample (40 B per index taken from its end); NULL allocates.
 */
int verify_claim(sf_circuit_t *c, const double *claimed, uint64_t k, uint64_t index_seed, double f1,
                 uint64_t path_seed, double delta, uint32_t flags, void *hip_stream, void *workspace,
                 size_t workspace_bytes, double *f_e, int *passed);

/* ------------------------------------------------------------------ */
/* Serving: jobs arrive at any time and share one GPU.                 */
/* ------------------------------------------------------------------ */
#define SF_PENDING 1   /* server_poll: the job has not finished yet */

typedef struct sf_server sf_server_t;   /* opaque */

/* One request: circuit, cut (0 = choose_cut), host bitstrings, fidelity f.
 * f >= 1 runs all 2^k paths; 0 < f < 1 runs sample_paths(k, f, path_seed)
 * (Section 3, Eq. (fid)).  The server copies everything it needs. */
typedef struct {
    int rows, cols;
    const sf_gate_t *gates;
    size_t n_gates;
    uint64_t block_a_mask;
    const uint64_t *bitstrings;
    size_t n_bits;
    double f;
    uint64_t path_seed;
    uint32_t flags;          /* 0 or SF_FP64_SWEEPS */
} sf_job_t;

typedef struct {
    double t_submit, t_admit, t_done;   /* seconds since server_create; t_submit is taken on entry
                                           to server_submit */
    uint64_t n_paths;
    uint32_t k;
    uint32_t chunks;                    /* path chunks run so far */
    int status;                         /* SF_PENDING, SF_OK or an error code */
} sf_job_info_t;

typedef struct {
    uint64_t arena_bytes, peak_bytes, in_use_bytes;
    uint64_t chunks;                    /* path chunks run */
    uint32_t max_concurrent_chunks;     /* most chunks in flight at once */
    uint32_t waiting, active;           /* jobs not yet admitted / admitted and unfinished */
} sf_server_stats_t;

/*
 * server_create: a serving runtime over one device-memory arena of
 * arena_bytes (caller memory `arena`, or NULL to let the server allocate it)
 * with n_workers workers (1..16), each owning a HIP stream of default
 * priority, and one thread that prepares submitted jobs (cut, path sample,
 * memory estimate).  A job is admitted when its memory (bitstrings, FP64
 * partial sums and a run_paths workspace, in the form of Section 9's M_proc)
 * fits in the arena; jobs that do not fit wait (later, smaller ones may
 * pass).  Admitted jobs are worked on in chunks of chunk_paths paths (0 =
 * 4096), one chunk per job at a time; a free worker takes the next chunk of
 * the admitted job the policy names (server_set_policy), so jobs admitted
 * while others run start on the next free worker and their kernels overlap
 * on the device.  Partial sums stay on the device until the job's last chunk.
 */
int server_create(size_t arena_bytes, void *arena, uint32_t n_workers, uint64_t chunk_paths,
                  sf_server_t **out);
/* server_submit: validate and copy a job (gate list, bitstrings) and enqueue it; returns at
 * once.  The cut, path sample and memory estimate are made on the server's preparation
 * thread; a job whose preparation fails (e.g. a bitstring outside the grid) finishes with that
 * error, which server_poll returns.  SF_ERR_OOM at once if even the smallest slice such a job
 * can have (bitstrings, FP64 sums, a 256 MiB workspace) exceeds the arena. */
int server_submit(sf_server_t *s, const sf_job_t *job, uint64_t *job_id);

/* Which admitted job a free worker serves next (server_set_policy):
 *   SF_SERVE_OLDEST_FIRST  the earliest admitted job with paths left (default): each job keeps
 *                          one worker from admission to completion, later jobs use the rest;
 *   SF_SERVE_ROUND_ROBIN   the admitted jobs in turn;
 *   SF_SERVE_LEAST_WORK    the job with the least remaining planned work (sweep and gather
 *                          bytes of its chunks, planned without device work). */
#define SF_SERVE_OLDEST_FIRST 0u
#define SF_SERVE_ROUND_ROBIN  1u
#define SF_SERVE_LEAST_WORK   2u
int server_set_policy(sf_server_t *s, uint32_t policy);
/* server_poll: SF_PENDING while running; SF_OK when done (copies 2*n_bits doubles
 * into amps if not NULL), or the job's error code. */
int server_poll(sf_server_t *s, uint64_t job_id, double *amps, sf_job_info_t *info);
/* server_release: forget a finished job and its host result. */
int server_release(sf_server_t *s, uint64_t job_id);
/* server_drain: block until every submitted job has finished. */
int server_drain(sf_server_t *s);
int server_stats(sf_server_t *s, sf_server_stats_t *out);
/* server_destroy: finish running chunks, stop the workers, free the server. */
int server_destroy(sf_server_t *s);
/* Message for the last server_* error on the calling thread. */
const char *server_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SFPATH_H */
