// Host-side launchers of the HIP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>

#include "sf_device.hpp"

namespace sf {

// Largest number of register qubits a pass kernel is instantiated for.  The
// op interpreter keeps about two copies of the tile in registers, so 2^5
// complex64 (2^4 complex128) amplitudes per lane leave room for 3 waves/SIMD.
constexpr int kMaxRegBits = 5;
constexpr int kMaxRegBitsF64 = 4;

// Stream one pass over a block state (see PassArgs).  R = register bits
// (0..kMaxRegBits), fp64 selects complex128 states.
// flips: the program holds PO_PFLIP_* ops (selects the kernel variant that has code for them)
// zskip: leave the amplitudes in the source's zero subspace (PassArgs::n_zero) unread, where a
// variant for (fp64, R, flips) exists; otherwise the list is ignored
hipError_t launch_pass(bool fp64, int R, bool flips, bool zskip, const PassArgs &a, unsigned grid, hipStream_t s);
// Two independent passes of the same kernel variant in one launch (grid0 + grid1 workgroups).
hipError_t launch_pass_pair(bool fp64, int R, bool flips, bool zskip, const PassArgs &a0, unsigned grid0,
                            const PassArgs &a1, unsigned grid1, hipStream_t s);

// A run of small dependent passes of one kernel variant in one cooperative (all workgroups
// resident) launch: n_phases ChainPhase entries from device memory, a grid barrier between
// phases on the 64-bit counter *count, which the call zeroes once and which only grows: base is
// what the call's earlier chains added to it ((phases - 1) * grid each).  A barrier wait that
// does not end sets bit 1 of *err and lets the kernel finish (the call then fails), so the launch
// always ends.  grid must not exceed chain_max_grid.
hipError_t launch_pass_chain(bool fp64, int R, bool flips, bool zskip, const PassArgs *args, const ChainPhase *phases,
                             uint32_t n_phases, uint64_t *count, uint64_t base, int *err, unsigned grid, hipStream_t s);
// Largest grid of launch_pass_chain for that variant whose workgroups are all resident at once.
hipError_t chain_max_grid(bool fp64, int R, bool flips, bool zskip, unsigned *grid);
// Whether launch_pass_chain runs that variant with zero-subspace skipping (otherwise it ignores
// PassArgs::n_zero, which only ever costs reads).
bool chain_zskip(bool fp64, int R, bool flips);

// Dense 4-qubit block on matrix cores (complex64 states only).
hipError_t launch_dense(const DenseArgs &a, unsigned grid, hipStream_t s);

// Gather + FP64 path sum for one leaf batch.
hipError_t launch_gather(bool fp64, const GatherArgs &g, hipStream_t s);

// Fold of the last tree levels + FP64 path sum for one batch of the level it reads (see
// FoldArgs); nb = path bits decided by the folded levels (1..5).  g.order and g.child_mask must
// be given.
hipError_t launch_fold(bool fp64, int nb, const FoldArgs &g, hipStream_t s);
// General fold (GFoldArgs) + FP64 path sum for one batch of the level it reads; nb = path bits
// decided by the folded levels (1..kMaxGFoldBits).  g.order and g.child_mask must be given.
constexpr int kMaxGFoldBits = 4;
hipError_t launch_gfold(bool fp64, int nb, const GFoldArgs &g, hipStream_t s);
// Fold of G (1..3) trailing crossing iSWAPs into the gather (FoldIswapArgs).
hipError_t launch_fold_iswap(bool fp64, int G, const FoldIswapArgs &g, hipStream_t s);

// key[i] = pext(x[i], mask) (32-bit).
hipError_t launch_key(const uint32_t *x, uint64_t n, uint32_t mask, uint32_t *key, hipStream_t s);

// *count += number of distinct values in the sorted array keys[0..n).
hipError_t launch_count_runs(const uint32_t *keys, uint64_t n, int *count, hipStream_t s);

// Rejection-sampling decisions for a batch of n FP64 complex amplitudes (see accept_kernel):
// flag[j] (0/1) and excess[j] per candidate, then the indices of accepted candidates in
// ascending order into accepted, their number into *n_accepted (device), and the sum of excess
// into *excess_sum (device).  temp: reject_temp_bytes(n) bytes.
hipError_t reject_temp_bytes(uint64_t n, size_t *bytes);
hipError_t launch_accept(const double *amps, uint64_t n, double scale, uint64_t seed, int basic, uint8_t *flag,
                         double *excess, uint32_t *accepted, uint64_t *n_accepted, double *excess_sum,
                         void *temp, size_t temp_bytes, hipStream_t s);

// Per-block partial sums (4 doubles per block: Re and Im of sum conj(a) b, sum |a|^2,
// sum |b|^2) over n complex FP64 pairs; b may be NULL.  partial: 4 * blocks doubles.
hipError_t launch_overlap(const double *a, const double *b, uint64_t n, double *partial, unsigned blocks,
                          hipStream_t s);

// x_A = pext(x, mask_a), x_B = pext(x, mask_b) per bitstring; *bad is set to
// 1 if some bitstring has bits outside `all`.
hipError_t launch_pext(const uint64_t *bits, uint64_t n, uint64_t mask_a, uint64_t mask_b,
                       uint64_t all, uint32_t *xa, uint32_t *xb, int *bad, hipStream_t s);

// order = indices 0..n-1 sorted by keys[i] (stable radix sort over key_bits bits); keys_sorted
// and idx are n-entry scratch arrays, temp a scratch area of sort_by_key_temp_bytes(n).
hipError_t sort_by_key_temp_bytes(uint64_t n, size_t *bytes);
hipError_t launch_order_by_key(const uint32_t *keys, uint32_t *keys_sorted, uint32_t *idx, uint32_t *order,
                               uint64_t n, int key_bits, void *temp, size_t temp_bytes, hipStream_t s);

// Fill n doubles with zero (a kernel, so it can also sit inside a captured graph).
hipError_t launch_fill_zero(double *p, uint64_t n, hipStream_t s);
// Row masks of the last passes before the path sum (PassArgs::row_mask): set bit
// (x_i & keep) | m for every bitstring i and every m inside spread (at most 8 bits).
hipError_t launch_mark_rows(const uint32_t *xh, uint64_t n, uint32_t keep, uint32_t spread, uint32_t *bitmap,
                            hipStream_t s);
// *count += set bits of words[0 .. n).
hipError_t launch_count_bits(const uint32_t *words, uint64_t n, unsigned long long *count, hipStream_t s);
// Streaming read of the first bytes (a power of two, at least 16) of buf, reps times (read_bandwidth).
hipError_t launch_read_probe(const void *buf, uint64_t bytes, uint32_t reps, unsigned grid, float *sink, hipStream_t s);
hipError_t launch_fill_zero_i32(int *p, uint64_t n, hipStream_t s);

}  // namespace sf
