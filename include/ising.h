/*
 * ising.h — C ABI of the MI355X (gfx950) checkerboard Metropolis library for the periodic
 * 2D Ising model (Yang et al., "High Performance Monte Carlo Simulation of Ising Model on TPU
 * Clusters", arXiv 1903.11714).
 *
 * Common rules for every entry point:
 *   - All functions are extern "C", return an int status (ISING_OK = 0, negative on error)
 *     and never throw.
 *   - Device pointers are HIP device allocations owned by the caller; the library never
 *     allocates, frees or keeps them.  Work is enqueued on `stream` (a hipStream_t, NULL for
 *     the default stream) and the call returns without synchronising.
 *   - Arguments are validated before anything is enqueued; ISING_EINVAL means nothing ran.
 *     ISING_EHIP means a HIP call failed; ising_last_error() returns its text.
 *   - Spin lattices hold +1 / -1 only (int8 layout) or the packed bit form of such a lattice.
 *     Other byte values give unspecified (but memory-safe) results.
 *   - L is the linear size of a square periodic lattice: L % 32 == 0, 32 <= L <= 2^20 (Sec. 3:
 *     any L x L torus; the kernels take 64-column groups, and a row whose length is an odd multiple
 *     of 32 ends in a half group of 32 columns).
 *   - Library state is process-wide: the options below (each an atomic value; every valid setting
 *     gives the same results, so a setting that races a launch is harmless) and the batched form's
 *     tuned schedules and captured graphs (guarded by a mutex held for the whole of each batch
 *     call), and one stream-ordered memory pool per device (created once under a mutex).
 *     ising_last_error is per thread.
 *   - Traced sweeps (a non-NULL trace_ME on ising_sweep, ising_sweep_fmt, ising_sweep_fused and
 *     ising_sweep_packed) take 512 KiB of device memory from that pool for the call, in stream
 *     order (hipMallocFromPoolAsync, then hipFreeAsync after the call's last launch), so calls on
 *     different streams never share it.  Their workgroups add (M, E) into 64 spread cache lines per
 *     launch instead of two words; one small kernel per 64 traced launches writes the sums into
 *     trace_ME.  The trace is complete once the stream reaches the end of the call.
 *
 * Lattice conventions (Sec. 3, Sec. 3.1, Sec. 3.2 of the paper):
 *   int8 layout: row-major L x L bytes, sigma[r][c] at offset r * L + c, periodic in r and c.
 *   colour of (r, c): (r + c) & 1; 0 = black, 1 = white.  A sweep updates every white site
 *   and then every black site (Sec. 3.1: alternate the two colours, white first).
 *   Acceptance (Sec. 3.2, Algorithm 1): a site with s = sigma * nn <= 0 flips; otherwise it
 *   flips iff its 32-bit uniform x is below T_s = ceil(2^32 exp(-2 beta s)), s in {2, 4}.
 *   The uniform of site (r, c) in sweep t: j = c >> 1, g = j >> 5, i = j & 31,
 *   p = 8 * (0, 2, 1, 3)[i & 3] + (i >> 2); bit 31 - k of x is bit p of word k & 3 of
 *   Philox4x32-10(key = (seed & 0xffffffff, seed >> 32), counter = (g, r, t, 2 (k >> 2) + q)).
 */
#ifndef ISING_H
#define ISING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ISING_OK = 0,
    ISING_EINVAL = -1,      /* invalid argument; nothing was enqueued        */
    ISING_EHIP = -2,        /* a HIP runtime call or kernel launch failed      */
    ISING_EUNSUPPORTED = -3 /* valid request this build or device cannot serve */
};

/* Hot start (the paper leaves the initial configuration open; Sec. 3.2 takes it as input):
 * spins[r * L + c] = -1 iff bit (c & 31) of word ((c >> 5) & 3) of
 * Philox4x32-10(key(seed), counter = (c >> 7, r, 0, 0x80000000)) is set, else +1.
 * spins: device int8[L * L], written completely. */
int ising_init(int8_t* spins, int64_t L, uint64_t seed, void* stream);

/* Cold start: every spin set to `value` (+1 or -1).  spins: device int8[L * L]. */
int ising_fill(int8_t* spins, int64_t L, int value, void* stream);

/* n_sweeps checkerboard Metropolis sweeps in place (Sec. 3.1 eq. 1, Sec. 3.2 Algorithm 1),
 * sweep indices t = sweep_offset .. sweep_offset + n_sweeps - 1 (the counter word of the
 * random numbers, so runs split into chunks reproduce an unsplit run bit for bit).
 *   spins     device int8[L * L], updated in place.
 *   beta      inverse temperature, finite and >= 0, or +inf (zero temperature).
 *   n_sweeps  >= 0;  sweep_offset + n_sweeps <= 2^32.
 *   trace_ME  device int64[2 * n_sweeps] receiving (M, E) after every sweep, or NULL.
 *             M = sum of spins, E = -sum over the 2 L^2 nearest-neighbour bonds of
 *             sigma_i sigma_j (Sec. 3 Hamiltonian with J = 1, mu = 0; Sec. 4.1 m = M / N). */
int ising_sweep(int8_t* spins, int64_t L, double beta, int64_t n_sweeps, uint64_t seed,
                uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* The same chain with low-precision acceptance (the paper's bfloat16 experiment, Sec. 4.1):
 *   fmt 0 = exact (identical to ising_sweep), 1 = bfloat16, 2 = IEEE half.
 * A site with s > 0 flips iff u < p, where p = exp(-2 beta s) rounded to nearest-even in fmt and
 * u = (top 16 bits of the site's exact-chain uniform) / 2^16 rounded toward zero in fmt.  Both
 * chains use the same random numbers; this one is the exact chain with the thresholds of
 * ising_thresholds_fmt. */
int ising_sweep_fmt(int8_t* spins, int64_t L, double beta, int fmt, int64_t n_sweeps, uint64_t seed,
                    uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* ising_sweep_fmt with both colours of a sweep -- and by default two whole sweeps -- in ONE pass
 * over the lattice (Sec. 3.1: given one colour, the other colour's sites are independent, so the
 * black sites of a row can be updated as soon as the white sites of the rows around it are, and
 * the next sweep's white sites of a row as soon as the black sites around it are).  Each pass
 * reads one L x L buffer and writes the other:
 *   scratch   device int8[L * L], 16-byte aligned, disjoint from spins; its contents on return
 *             are unspecified.  The caller owns it.
 * On return `spins` holds the lattice after n_sweeps sweeps, bit-identical to ising_sweep_fmt
 * with the same arguments, and so is trace_ME.  Passes alternate spins -> scratch -> spins, an
 * even number of them; an odd count runs its first sweep in place.  Option "fused_sweeps" sets
 * the sweeps per pass (2 by default, 1).  Up to L = 16384 a pass gives each row to one workgroup
 * (one thread per 64-column group), and the two-sweep pass spaces its four updates three rows apart,
 * so that two consecutive steps are independent and their still-tied words are settled together
 * (option "fused_pairs"); above L = 16384 the two-sweep pass runs in column bands of one wave each
 * (62 own groups and one recomputed group on either side; option "fused_bands" moves the switch).
 * The one-sweep pass needs a whole row per workgroup: above L = 65536 it is not available
 * (fused_sweeps = 1 then sweeps in place as ising_sweep_fmt).  When L % 64 != 0 every sweep runs in
 * place as in ising_sweep_fmt (scratch unused).  Returns ISING_EINVAL for the checks of
 * ising_sweep_fmt, for a null, misaligned or overlapping scratch. */
int ising_sweep_fused(int8_t* spins, int8_t* scratch, int64_t L, double beta, int fmt, int64_t n_sweeps,
                      uint64_t seed, uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* ising_sweep_fused for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the second lattice buffer and the spread sets of
 * a traced call are the library's own static device array of 64 MiB + 512 KiB, so L * L <= 2^26
 * (L <= 8192); larger L returns ISING_EINVAL.  The call allocates and frees nothing.  Every call on one GPU shares that GPU's array (each GPU holds
 * its own until the process ends); calls that overlap on one GPU, on different streams or threads,
 * race and give unspecified results.  Arguments, results and errors otherwise as ising_sweep_fused. */
int ising_sweep_fused_static(int8_t* spins, int64_t L, double beta, int fmt, int64_t n_sweeps, uint64_t seed,
                             uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* One sweep with sweep index t (< 2^32) out of place: dst = the sweep of src (both device
 * int8[L * L], 16-byte aligned, disjoint; src is not modified).  out_ME: NULL or device int64[2]
 * receiving (M, E) of dst.  For a caller that manages its own pair of buffers (a captured graph
 * of alternating steps, say).  Above L = 65536, or when L % 64 != 0: a device copy, then the two
 * half-sweeps on dst. */
int ising_sweep_fused_step(const int8_t* src, int8_t* dst, int64_t L, double beta, int fmt, uint64_t seed,
                           uint64_t t, int64_t* out_ME, void* stream);

/* Two sweeps, t and t + 1 (t + 1 < 2^32), in one pass out of place: dst = src after both (same
 * buffers and conventions as ising_sweep_fused_step).  out_ME: NULL or device int64[4] receiving
 * (M, E) after sweep t, then after sweep t + 1.  Above L = 16384 the pass runs in column bands;
 * when L % 64 != 0: a device copy, then the four half-sweeps on dst. */
int ising_sweep_fused_pair(const int8_t* src, int8_t* dst, int64_t L, double beta, int fmt, uint64_t seed,
                           uint64_t t, int64_t* out_ME, void* stream);

/* One colour update (half of a sweep) for colour q in {0, 1} with sweep index t.
 * Same arguments as ising_sweep otherwise; t < 2^32. */
int ising_half_sweep(int8_t* spins, int64_t L, double beta, uint64_t seed, uint64_t t, int q,
                     void* stream);

/* out_ME: device int64[2] receiving (M, E) of the lattice (definitions as above, Sec. 3 and
 * Sec. 4.1).  Exact integer sums; the result does not depend on the launch order. */
int ising_observables(const int8_t* spins, int64_t L, int64_t* out_ME, void* stream);

/* ---- Three dimensions -----------------------------------------------------------------------
 * The d-dimensional hypercubic lattice of Sec. 3 at d = 3, with the checkerboard colouring of
 * Fig. 1 extended to three dimensions.  spins: device int8[L * L * L], 16-byte aligned, site
 * (z, y, x) at index (z L + y) L + x, values +1 / -1; L a power of two, 64 <= L <= 2048.
 * Colour q = (x + y + z) mod 2; a sweep updates white (q = 1) then black.  nn = sum of the six
 * neighbours, s = sigma nn; a site flips iff s <= 0 or its uniform x < T_s = ceil(2^32
 * exp(-2 beta s)) for s = 2, 4, 6.  The random numbers are those of the square lattice with row
 * index r = z L + y (Philox counter (x >> 6, z L + y, t, 2m + q), hot start as ising_init on L^2
 * rows).  E = -sum over the 3 L^3 bonds of sigma_i sigma_j (each site's +x, +y, +z neighbour).
 * Same conventions and error codes as the square-lattice calls. */
int ising3_init(int8_t* spins, int64_t L, uint64_t seed, void* stream);
int ising3_fill(int8_t* spins, int64_t L, int value, void* stream);
int ising3_sweep(int8_t* spins, int64_t L, double beta, int64_t n_sweeps, uint64_t seed, uint64_t sweep_offset,
                 int64_t* trace_ME, void* stream);

/* ising3_sweep with both colours of a sweep in ONE pass over the lattice, out of place (as
 * ising_sweep_fused on the square lattice): each pass reads one L^3 buffer and writes the other.
 *   scratch   device int8[L^3], 16-byte aligned, disjoint from spins; contents on return
 *             unspecified; caller-owned.
 * On return `spins` holds the lattice after n_sweeps sweeps, bit-identical to ising3_sweep, and
 * so is trace_ME.  Sweeps go spins -> scratch -> spins in pairs; an odd count runs its first
 * sweep in place.  ISING_EINVAL for the checks of ising3_sweep and a null, misaligned or
 * overlapping scratch. */
int ising3_sweep_fused(int8_t* spins, int8_t* scratch, int64_t L, double beta, int64_t n_sweeps, uint64_t seed,
                       uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* One sweep with index t (< 2^32) out of place: dst = the sweep of src (device int8[L^3] each,
 * 16-byte aligned, disjoint; src unchanged).  out_ME: NULL or device int64[2] receiving (M, E)
 * of dst. */
int ising3_sweep_fused_step(const int8_t* src, int8_t* dst, int64_t L, double beta, uint64_t seed, uint64_t t,
                            int64_t* out_ME, void* stream);
int ising3_half_sweep(int8_t* spins, int64_t L, double beta, uint64_t seed, uint64_t t, int q, void* stream);
int ising3_observables(const int8_t* spins, int64_t L, int64_t* out_ME, void* stream);
/* out[0..2] = T_2, T_4, T_6 (host). */
int ising3_thresholds(double beta, uint64_t out[3]);

/* 1-bit layout of the cubic lattice: the square lattice's packed layout over the L^2 rows
 * r = z L + y.  planes: device uint32[L^3 / 32]; word (q L^2 + r) (L / 64) + g holds the colour-q
 * sites of row r with j = x >> 1 in [32 g, 32 g + 32), site i at bit 8 (0, 2, 1, 3)[i & 3] + (i >> 2);
 * colour q of row (z, y) sits at column parity (q + y + z) mod 2; a set bit is spin -1.  The same
 * chain as the int8 calls (bit-identical spins and (M, E)). */
int ising3_pack(const int8_t* spins, int64_t L, uint32_t* planes, void* stream);
int ising3_unpack(const uint32_t* planes, int64_t L, int8_t* spins, void* stream);
int ising3_init_packed(uint32_t* planes, int64_t L, uint64_t seed, void* stream);
int ising3_sweep_packed(uint32_t* planes, int64_t L, double beta, int64_t n_sweeps, uint64_t seed,
                        uint64_t sweep_offset, int64_t* trace_ME, void* stream);
int ising3_half_sweep_packed(uint32_t* planes, int64_t L, double beta, uint64_t seed, uint64_t t, int q,
                             void* stream);
int ising3_observables_packed(const uint32_t* planes, int64_t L, int64_t* out_ME, void* stream);

/* ---- 1-bit packed layout -----------------------------------------------------------------
 * planes: device uint32[ising_packed_words(L)] = uint32[2 L G], G = ceil(L / 64): two colour
 * planes of L rows x G words each (L * L / 32 words when L % 64 == 0).  Word (q * L + r) * G + g
 * holds the colour-q sites of row r with j = c >> 1 in [32 g, 32 g + 32); site i = j & 31 sits at
 * bit 8 * (0, 2, 1, 3)[i & 3] + (i >> 2) (the bit position its uniform uses); a set bit is spin -1.
 * When L % 64 == 32 the last word of each row holds sites 0 .. 15 only (bits 0 .. 3 of each byte);
 * its other bits are zero. */

/* Number of uint32 words of the packed layout for L (2 L ceil(L / 64)), or ISING_EINVAL. */
int64_t ising_packed_words(int64_t L);

int ising_pack(const int8_t* spins, int64_t L, uint32_t* planes, void* stream);
int ising_unpack(const uint32_t* planes, int64_t L, int8_t* spins, void* stream);

/* Cold start in the packed layout: every spin `value` (+1 or -1). */
int ising_fill_packed(uint32_t* planes, int64_t L, int value, void* stream);

/* Hot start written directly in the packed layout (equals ising_pack of ising_init). */
int ising_init_packed(uint32_t* planes, int64_t L, uint64_t seed, void* stream);

/* The same chain as ising_sweep on the packed layout: identical spins after every sweep and
 * the same (M, E) trace.  Arguments as for ising_sweep. */
int ising_sweep_packed(uint32_t* planes, int64_t L, double beta, int64_t n_sweeps,
                       uint64_t seed, uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* ising_sweep_fmt on the packed layout. */
int ising_sweep_packed_fmt(uint32_t* planes, int64_t L, double beta, int fmt, int64_t n_sweeps,
                           uint64_t seed, uint64_t sweep_offset, int64_t* trace_ME, void* stream);

/* One colour update on the packed layout (as ising_half_sweep). */
int ising_half_sweep_packed(uint32_t* planes, int64_t L, double beta, uint64_t seed, uint64_t t,
                            int q, void* stream);

/* (M, E) of a packed lattice into device int64[2]. */
int ising_observables_packed(const uint32_t* planes, int64_t L, int64_t* out_ME, void* stream);

/* ---- batched replicas ----------------------------------------------------------------------
 * Many small independent lattices (L = 32, or L % 64 == 0 up to 512), each with its own beta and
 * seed, run in ONE persistent launch (captured in a hipGraph and replayed on `stream`).  Each
 * replica is held in LDS for every sweep of the run, by one workgroup or, when it is split, by 2,
 * 4 or 8 slabs of at least 16 rows (so large replicas do not hold the whole run on one compute
 * unit).  A slab also holds and updates d rows beyond either edge, so it trades its outer d rows
 * with its neighbours through the workspace only every d colour updates (d = 1, 2 or 4).  With
 * a split, slabs and whole replicas are packed into one or two work lists per compute unit,
 * balanced by size (largest first onto the least loaded list), one workgroup per list.  Every replica is the single-lattice chain of its (L, beta, seed):
 * identical spins and (M, E) to ising_sweep_packed on that lattice alone, for every split (the
 * paper's per-(L, T) Markov chains, Sec. 4.1). */
typedef struct {
    int64_t L;       /* linear size: 32, or a multiple of 64 up to 512 */
    double beta;     /* finite >= 0 or +inf */
    uint64_t seed;   /* Philox key of this replica */
} ising_replica_t;

/* Device workspace size for the batch (replica table, every replica's packed lattice, the slab
 * table and the row-exchange areas), or ISING_EINVAL.  replicas: host array of n entries. */
int64_t ising_batch_workspace_bytes(const ising_replica_t* replicas, int64_t n);

/* n_therm + n_meas sweeps of every replica (sweep indices sweep_offset ..), all in one launch.
 *   fmt        acceptance format as for ising_sweep_fmt (0 exact, 1 bfloat16, 2 half).
 *   start      0 = hot start from each seed, 1 = cold start (all +1), 2 = continue from the
 *              lattices left in `workspace` by a previous call with the same replicas,
 *              3 = cold start where beta > beta_c = ln(1 + sqrt 2) / 2 (ordered phase, where a
 *              hot start would only coarsen slowly), hot start elsewhere.
 *   workspace  device buffer of ising_batch_workspace_bytes bytes (caller-owned, 16-byte aligned);
 *              holds the lattices between calls.
 *   trace_ME   device int64[n * n_meas * 2] (replica-major (M, E) after every measurement sweep)
 *              or NULL.
 *   moments    device double[n * 5]: per replica <|m|>, <m^2>, <m^4>, <e>, <e^2> over the
 *              measurement sweeps, summed in FP64 in sweep order, or NULL.
 * n_therm + n_meas < 2^31.
 * The schedule -- workgroup size (256, 512 or 1024 threads), split (no split, or slabs of at most
 * 65536, 32768 or 16384 sites), d and lists per compute unit -- is picked once per set of replica
 * sizes by timing the candidates on the table itself (options "batch_threads",
 * "batch_slab_sites", "batch_depth" and "batch_lists_per_cu" fix them);
 * every schedule gives identical results.  The first call for a new set of sizes synchronises
 * for that timing; every other call returns without synchronising.  The run is captured once per
 * plan (workspace address and layout, schedule) into a hipGraph; the per-call values (start mode,
 * sweep counts, trace and moments pointers) are written into the workspace by a small kernel on
 * `stream` ahead of the graph, so repeated calls replay one graph.  At most 8 plans stay captured;
 * making a ninth waits for the latest run of the least recently used one (that run only, not the
 * device) before releasing it.  A split schedule is used only if all its workgroups fit on the GPU at once
 * (slabs wait for their neighbours' rows); its waits are bounded, and a run in which one gave up
 * (possible only if other work keeps its workgroups off the GPU, e.g. two batch runs at once on
 * different streams) writes NaN moments for the replicas concerned. */
int ising_batch_run(const ising_replica_t* replicas, int64_t n, int64_t n_therm, int64_t n_meas,
                    uint64_t sweep_offset, int fmt, int start, void* workspace, int64_t workspace_bytes,
                    int64_t* trace_ME, double* moments, void* stream);

/* The schedule ising_batch_run picked for this set of replica sizes: out[0] = threads per
 * workgroup, out[1] = split target in sites per slab (-1: no split), out[2] = colour updates
 * between exchanges of a split replica, out[3] = work lists per compute unit of a split
 * schedule.  Host pointers; returns ISING_EINVAL if no run has tuned this set of sizes yet. */
int ising_batch_schedule(const ising_replica_t* replicas, int64_t n, int64_t out[4]);

/* Replica j's lattice from the batch workspace as int8 rows (device int8[L_j * L_j]). */
int ising_batch_unpack(const void* workspace, int64_t n, int64_t j, int8_t* spins, void* stream);

/* ---- host helpers -------------------------------------------------------------------------- */

/* The two acceptance thresholds for beta: out[0] = T_2, out[1] = T_4 (each in [0, 2^32]),
 * T_s = ceil(2^32 exp(-2 beta s)).  Host pointer.  Sec. 3.2, Algorithm 1. */
int ising_thresholds(double beta, uint64_t out[2]);

/* Integer thresholds of the fmt acceptance: out[k] = R_s 2^16 with R_s the number of 16-bit
 * uniforms r whose rounded value is below the rounded probability (fmt 0: ising_thresholds). */
int ising_thresholds_fmt(double beta, int fmt, uint64_t out[2]);

/* FP64 moments of a traced chain (Sec. 4.1: m and the Binder cumulant need <m^2>, <m^4>):
 * out (device double[5]) = (<|m|>, <m^2>, <m^4>, <e>, <e^2>) over the n traced sweeps, with
 * m = M / n_sites and e = E / n_sites; the sums run in sweep order, so the result is
 * deterministic.  trace_ME: device int64[2 n] as written by ising_sweep. */
int ising_moments(const int64_t* trace_ME, int64_t n, int64_t n_sites, double* out, void* stream);

/* Launch-shape options of the int8 kernels, process-wide; results are bit-identical for every
 * valid setting (the random numbers depend only on site, sweep and colour).  Not thread-safe
 * against concurrent launches.
 *   "rows_per_lane"  rows each lane of a one-colour launch (int8 or packed) streams through:
 *                    0 = automatic (int8: the tallest up to 32 that leaves 2^18 lanes; packed: up
 *                    to 32 leaving 2^19 lanes, 4 at least), else a power of two in [2, 64]
 *                    (ignored for lattices it does not divide).
 *   "xcd_remap"      1 = hand each XCD one contiguous range of row strips (default), 0 = not.
 *   "nt_store"       1 = non-temporal stores of updated rows, 0 = ordinary stores (default).
 *   "staged"         1 = coalesced row loads and stores regrouped through LDS when L is a
 *                    multiple of 4096 (default), 0 = every lane reads its own 64 bytes.
 *   "batch_threads"  workgroup size of ising_batch_run: 0 = autotune (default), 256, 512, 1024.
 *   "batch_slab_sites"  ising_batch_run: split replicas into row slabs of at most this many sites
 *                    (a power of two from 1024 to 262144; slabs keep at least 16 rows, at most 8
 *                    per replica), -1 = never split, 0 = autotune (default).
 *   "batch_depth"    ising_batch_run: colour updates between row exchanges of a split replica
 *                    (1, 2 or 4), 0 = autotune (default).
 *   "batch_lists_per_cu"  ising_batch_run: work lists per compute unit of a split schedule (1 or
 *                    2), 0 = autotune (default).
 *   "fused_rows"     rows per workgroup strip of ising_sweep_fused: 0 = automatic, else an even
 *                    number in [2, 256].  The two-sweep pass with paired steps takes any such value
 *                    (its strips then hold that many rows or two fewer); the other passes ignore a
 *                    value that does not divide L.
 *   "fused_alternate" 1 = odd strips of ising_sweep_fused walk upwards (default), 0 = all down.
 *   "fused_bands"    two-sweep passes in column bands of one wave: 0 = above L = 16384 (default),
 *                    1 = from L = 4096, 2 = only above L = 65536 (rows wherever a whole row fits
 *                    one workgroup: up to 512 groups with paired steps, else one step per settle).
 *   "band_rows"      rows per strip of the band pass: 0 = automatic (a power of two in [8, 256]
 *                    chosen from the waves each SIMD would run), else a power of two in [2, 1024]
 *                    (ignored for lattices it does not divide).
 *   "fused_sweeps"   sweeps per pass of ising_sweep_fused: 2 (default) or 1.
 *   "fused_ties"     fused passes (two sweeps or one): 1 = the updates of a step are independent
 *                    and the words still tied after two Philox blocks are settled together
 *                    (default), 0 = each update settles its own words before the next one.
 *   "fused_pairs"    two-sweep passes of rows of at most 512 groups (L <= 32768): 1 = the four
 *                    updates of a step are three rows apart, and two steps share one edge exchange
 *                    and one settle of their still-tied words (default), 0 = two rows apart, one
 *                    step at a time (used only with "fused_ties" = 1).
 *   "packed_ties"    ising_sweep_packed / ising_half_sweep_packed (and the 3-D packed sweep, four
 *                    planes): 1 = each lane takes four rows at a time and their still-tied words are
 *                    settled together (default; used when the rows per lane are a multiple of 4),
 *                    0 = row by row.
 *   "ties3"          ising3_sweep / ising3_half_sweep: 1 = the two planes of each step share one
 *                    row exchange and their still-tied words are settled together (default),
 *                    0 = plane by plane.  ising3_sweep_fused / ising3_sweep_fused_step: 1 = each
 *                    step updates the white sites of planes z, z + 1 and the black sites of planes
 *                    z - 3, z - 2 and settles their still-tied words together (default), 0 = the
 *                    white sites of plane z, then the black sites of plane z - 1, each on its own.
 *   "planes3"        planes each workgroup of ising3_sweep (each lane of ising3_sweep_packed)
 *                    walks: 0 = automatic, else a power of two in [2, 256] (ignored for lattices it
 *                    does not divide). */
int ising_set_option(const char* name, int64_t value);
int ising_get_option(const char* name, int64_t* value);

/* Text of the most recent ISING_EHIP failure on this thread (empty if none). */
const char* ising_last_error(void);

/* Static text for a status code. */
const char* ising_strerror(int status);

/* Library version as major * 10000 + minor * 100 + patch. */
int ising_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
