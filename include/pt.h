/*
 * pt.h -- C ABI of libpt.so: replica-exchange Metropolis simulation of an
 * elastic bead-spring homopolymer on an AMD Instinct MI355X (gfx950).
 *
 * The method is the one of Gross, Janke and Bachmann, "Massively
 * parallelized replica-exchange simulations of polymers on GPUs" (Comput.
 * Phys. Commun.; arXiv:1107.3490):
 *   - model: truncated, shifted Lennard-Jones between all monomer pairs
 *     (Sec. 3.1, Eqs. 1-2) plus FENE bonds between chain neighbours (Eq. 3);
 *     total energy Eq. (4);
 *   - local update: a random monomer is displaced by a vector uniform in a
 *     cube (Sec. 3.2), accepted with the Metropolis probability (Eq. 5);
 *   - replica exchange between neighbouring temperatures (Sec. 3.3, Eq. 6);
 *   - per-sweep energy, end-to-end distance and radius of gyration (the
 *     kernel description of Sec. 3.4; Eq. 8).
 *
 * Arithmetic contract.  Every accept/reject and exchange decision equals,
 * bit for bit, the one taken by the FP64 reference order:
 *   r2   = fma(dz, dz, fma(dy, dy, dx*dx))
 *   e    = 0 if !(r2 < rc^2), else s2 = sig^2/r2, s6 = (s2*s2)*s2,
 *          e = fma(4 eps, s6*(s6-1), -E_LJ(rc))
 *   F    = +inf if !(y > 0), else ((-0.5 K) R) R * log(y),
 *          y = fma(-x, x, 1), x = (sqrt(r2) - r0)/R
 *   log  = argument reduction to [sqrt(1/2), sqrt(2)), s = f/(2+f), odd
 *          atanh series to s^21 (Horner, fma), e*ln2 split in two parts
 *   dE   = (pairwise tree over the zero-padded power-of-two bead range of
 *          e(new) - e(old), moved bead excluded) + (dF_left + dF_right)
 *   E    = (tree over rows i of the tree over j of [i<j<N] e(r2_ij))
 *          + (tree over bonds of F)
 *   accept move     iff dE <= 0 or beta*dE < -log(u)
 *   accept exchange iff D >= 0 or log(u) < D, D = (b_i - b_{i+1})(E_i - E_{i+1})
 * with the derived constants sig^2 = sigma*sigma, rc^2 = r_cut*r_cut,
 * E_LJ(rc) = (4 eps) * (s6*(s6-1)) at s2 = sig^2/rc^2.  Random numbers are
 * Philox4x32-10 (Salmon et al., SC'11), key = (seed lo, seed hi):
 *   move m of sweep t in stream slot g:  counters (m,t,g,0) -> w0..w3 and
 *   (m,t,g,1) -> v0;  k = floor(w0*N/2^32);  d_a = (((w_a+.5)2^-32)-.5)*edge;
 *   u = (v0+.5)2^-32;
 *   exchange of slots (i,i+1) of stream chain c at step e: counter (i,e,c,2).
 * PT_FP64 evaluates the pair terms in that order.  PT_MIXED evaluates the
 * bracket s6*(s6-1) of each pair in FP32 from r^2 formed in FP64 from the FP64
 * separation (r^2 clamped at the cutoff), sums the
 * differences of new and old brackets in FP32 as the same pairwise tree (so
 * every output is independent of the mapping) and scales the sum by 4 eps
 * (the shift E_LJ(rc) cancels in each difference), adds the FP64 bond terms
 * in FP64, and re-scores
 * in the FP64 order every decision that a rigorous error bound cannot settle;
 * its running energies carry that bound and are re-synchronised with the FP64
 * energy whenever an exchange decision needs it.  At the end of a sweep the running
 * energy is replaced by the FP64-order energy when its bound exceeds 2^-30
 * (PT_FP64, and PT_MIXED with PT_SCHED_FP64_ON_ACCEPT) or 2^-6 (PT_MIXED)
 * of max(1, |E|).
 *
 * Threading: a handle is not thread-safe.  Separate handles on separate
 * streams are independent.  All device work of a handle is enqueued on the
 * stream given to pt_init.
 *
 * Errors: every int-returning call returns PT_OK (0) or a negative code;
 * pt_last_error() gives a message (thread-local).  Asynchronous device
 * faults, and a persistent run whose blocks stopped waiting for each other
 * after a timeout, surface as PT_EHIP at the next call that synchronises.
 */
#ifndef PT_H
#define PT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
#define PT_API extern "C" __attribute__((visibility("default")))
#else
#define PT_API __attribute__((visibility("default")))
#endif

enum pt_status {
    PT_OK = 0,
    PT_EINVAL = -1,        /* bad argument or model/config value                 */
    PT_EDOMAIN = -2,       /* an initial bond at or beyond r0 +- R (Eq. 3)       */
    PT_ENOMEM = -3,        /* workspace smaller than pt_workspace_bytes()        */
    PT_EHIP = -4,          /* a HIP runtime call failed                          */
    PT_ESTATE = -5,        /* call not valid in the handle's current state       */
    PT_EUNSUPPORTED = -6   /* chain longer than the kernels support (N > 2048),
                              PT_MAP_LANE with PT_MIXED, or PT_MAP_PACK2/4 with
                              a layout other than B <= 2, W = 1                  */
};

enum pt_precision { PT_FP64 = 0, PT_MIXED = 1 };

/* Model parameters (Sec. 3.1; step_edge is the displacement cube edge of
 * Sec. 3.2, the paper's value being 0.02).  All must be finite and > 0. */
typedef struct pt_model {
    double epsilon, sigma, r_cut, fene_k, fene_R, fene_r0, step_edge;
} pt_model;

/* A batch of independent chains, each with its own temperature ladder.
 * Host arrays are read during pt_init only (copied). */
typedef struct pt_config {
    int32_t n_chains;               /* >= 1                                           */
    const int32_t *n_beads;         /* [n_chains], 2 <= N <= 2048                      */
    const int32_t *n_slots;         /* [n_chains], >= 1 (temperatures per chain)       */
    const double *beta;             /* [sum R_c], finite, >= 0; chain-major            */
    const double *coords;           /* [sum_c R_c*N_c*3] starting conformation of every
                                       slot, chain-major, bead-major, xyz (AoS)        */
    const uint32_t *stream_chain;   /* [n_chains] chain id in exchange counters, or NULL
                                       (= position in the batch)                       */
    const uint32_t *stream_slot0;   /* [n_chains] stream id of each chain's slot 0, or
                                       NULL (= running slot offset)                    */
    uint64_t seed;                  /* Philox key                                      */
    int32_t precision;              /* PT_FP64 or PT_MIXED                             */
    int32_t exchange_every;         /* exchange step after sweep t if (t+1)%k == 0;
                                       0 = only explicit pt_exchange()                 */
    int64_t series_capacity;        /* sweeps of (E, Ree^2, Rg^2) per slot kept on the
                                       device; 0 = none                                */
    int64_t log_capacity;           /* sweeps of accept bits and exchange outcomes kept
                                       on the device; 0 = none                         */
    int32_t schedule;               /* PT_SCHED_AUTO, PT_SCHED_PER_SWEEP,
                                       PT_SCHED_PERSISTENT or PT_SCHED_FLOW (same
                                       results), optionally | PT_SCHED_FULL_ENERGY
                                       and | PT_SCHED_FP64_ON_ACCEPT                 */
    const int32_t *mapping;         /* [n_chains] 16*B + W (beads per lane B in
                                       {1,2,4,8}, wavefronts per replica W in {1,2,4},
                                       64*W*B >= N), optionally | PT_MAP_LANE,
                                       PT_MAP_PACK2 or PT_MAP_PACK4, or 0
                                       for the default; NULL = all default.  Results
                                       do not depend on it.                            */
} pt_config;

/* How pt_sweep runs a class of chains (chains with the same mapping).
 * PER_SWEEP: one sweep kernel launch per sweep, then an exchange kernel.
 * PERSISTENT: one launch for all n sweeps; every replica stays on the chip
 * and exchange attempts synchronise the two blocks of a pair only.  The
 * classes of one wavefront count W share that launch (each block runs its
 * chain's bead count per lane) as long as all their replicas fit on the
 * device at once; launches of different W follow one another.  A class that
 * does not fit takes FLOW if it has 1024 or more bead slots per replica
 * (64 W B), else PER_SWEEP.
 * FLOW: one launch for all n sweeps with as many blocks as fit; they take
 * (sweep, slot) tasks in order, each task sweeping one replica from device
 * memory, and the task that finishes an attempted pair's sweep second takes
 * the exchange decision; no block ever waits for a later task.
 * AUTO = PERSISTENT.  Every schedule gives the same results bit for bit. */
enum pt_schedule { PT_SCHED_AUTO = 0, PT_SCHED_PER_SWEEP = 1, PT_SCHED_PERSISTENT = 2, PT_SCHED_FLOW = 3 };

/* The paper's alternative designs, kept as measured alternatives (Sec. 3.4,
 * Sec. 4.2); results are unchanged bit for bit.
 * PT_SCHED_FULL_ENERGY (or-ed into config.schedule): every sweep ends with
 * the FP64-order energy E(C) of Eq. (4), recomputed from scratch, in place
 * of the running sum of the accepted moves' differences (which is otherwise
 * replaced only when its error bound has grown); the recorded E is then the
 * FP64-order energy of every sweep.
 * PT_MAP_LANE (or-ed into a chain's mapping code, precision PT_FP64 only):
 * one lane runs the whole sweep of one replica, 64 replicas per wavefront,
 * coordinates read from and written to device memory bead by bead (the
 * 16*B + W part then only fixes the storage layout); never persistent.
 * PT_SCHED_FP64_ON_ACCEPT (or-ed into config.schedule, PT_MIXED; no effect
 * with PT_FP64): every accepted move is also re-scored in the FP64 order,
 * so the running energy adds FP64-order differences only, is re-synchronised
 * at PT_FP64's threshold and is as accurate as PT_FP64's (the decisions are
 * the same either way); accepted moves then count as re-scored in
 * pt_observables. */
enum pt_ablation { PT_SCHED_FULL_ENERGY = 16, PT_SCHED_FP64_ON_ACCEPT = 32, PT_MAP_LANE = 0x100 };

/* Several replicas per wavefront for short chains (the occupancy question of
 * Sec. 4.2: a chain of 13 beads fills 13 of a wavefront's 64 lanes).
 * PT_MAP_PACK2 / PT_MAP_PACK4 (or-ed into a chain's mapping code, layouts
 * 16*B + 1 with B = 1 or 2, i.e. N <= 64 B; both precisions): two or four
 * replicas of the chain share a wavefront, 32 or 16 lanes each, every lane
 * holding 2 B or 4 B beads; the replicas keep the layout of 16*B + 1, so all
 * other calls treat the chain as mapped to 16*B + 1.  Sweeps run one launch per
 * sweep (never persistent); results are those of 16*B + 1 bit for bit. */
enum pt_map_pack { PT_MAP_PACK2 = 0x200, PT_MAP_PACK4 = 0x400 };

typedef struct pt_handle pt_handle;

/* Device workspace needed for (model, config), in bytes (256-byte aligned
 * start required).  Returns 0 and sets the error message on invalid input. */
PT_API size_t pt_workspace_bytes(const pt_model *model, const pt_config *config);

/* Validate, lay out the caller's device workspace, upload ladders and
 * coordinates, compute every starting energy in the FP64 order (Eq. 4) and
 * enqueue all of it on hip_stream (a hipStream_t; NULL = the null stream).
 * The workspace belongs to the caller, must outlive the handle and must not
 * be touched while the handle lives.  Synchronises the stream once.
 * Errors: PT_EINVAL, PT_EDOMAIN, PT_ENOMEM, PT_EUNSUPPORTED, PT_EHIP. */
PT_API int pt_init(const pt_model *model, const pt_config *config, void *d_workspace,
                   size_t ws_bytes, void *hip_stream, pt_handle **out);

/* Enqueue n sweeps (Sec. 3.2: one sweep = N attempted single-monomer moves
 * per slot), each followed by the per-sweep record and, when due, one
 * exchange step (Sec. 3.3).  Asynchronous.  n >= 0. */
PT_API int pt_sweep(pt_handle *h, int64_t n_sweeps);

/* Enqueue one exchange step (Eq. 6) now, advancing the exchange index e. */
PT_API int pt_exchange(pt_handle *h);

/* Synchronous: FP64-order energy E(C) (Eq. 4) of the conformation held by
 * each slot, [sum R_c] doubles, chain-major. */
PT_API int pt_energy(pt_handle *h, double *h_energy);

/* Energy of each slot's conformation (Eq. 4) by one of two methods,
 * synchronous, [sum R_c] doubles each:
 *   PT_ENERGY_FP64_ORDER: the FP64-order energy of pt_energy (the wavefronts
 *     of a conformation's block share its rows of pairs, one row per lane);
 *     h_bound gets the a-priori
 *     bound on |E - exact sum of the FP64 terms| that the kernels use;
 *   PT_ENERGY_PAIR_PER_THREAD: the paper's parallel energy (Sec. 3.4): the
 *     coordinates in LDS, every thread sums one pair per round, rows i and
 *     N-2-i sharing a round, then a reduction over threads; for even N the
 *     middle round takes its row once (the printed enumeration skips it).
 *     Not the FP64 order: E differs from it by rounding, and h_bound gets a
 *     rigorous bound on |E - exact sum of the same FP64 terms|.
 * h_bound and kernel_ms (HIP event time of the energy launches on the
 * handle's stream, ms) may be NULL.  Errors: PT_EINVAL, PT_EHIP. */
enum pt_energy_method { PT_ENERGY_FP64_ORDER = 0, PT_ENERGY_PAIR_PER_THREAD = 1 };
PT_API int pt_energy_method(pt_handle *h, int32_t method, double *h_energy, double *h_bound,
                            double *kernel_ms);

/* Observables and counters.  Every pointer may be NULL.  Synchronous.
 *   acc     [slots][5]: sweeps recorded, sum E, sum E^2, sum Rg^2, sum Ree^2
 *           (E is the running energy; Rg^2 per Eq. 8; Ree^2 = |r_N - r_1|^2)
 *   counts  [slots][7]: moves accepted, exchange attempts of pair (g,g+1),
 *           exchange accepts of pair (g,g+1), moves re-scored in FP64,
 *           exchange decisions that needed FP64 energies, moves attempted,
 *           sweeps that ended with a re-synchronisation of the running energy
 *   perm    [slots]: conformation held by each slot
 *   te      [2]: sweeps done t, exchange steps done e */
PT_API int pt_observables(pt_handle *h, double *acc, int64_t *counts, int32_t *perm, int64_t *te);

/* Zero the observable accumulators (after burn-in).  Asynchronous. */
PT_API int pt_reset_observables(pt_handle *h);

/* Synchronous copies of the state.
 *   pt_get_coords:  [sum_c R_c*N_c*3] conformations in their original order
 *                   (conformation q started in slot q), AoS;
 *   pt_get_running: running energy and its error bound per conformation. */
PT_API int pt_get_coords(pt_handle *h, double *h_coords);
PT_API int pt_get_running(pt_handle *h, double *h_energy, double *h_bound);

/* Synchronous copies of the recorded series and logs (rows since pt_init, at
 * most the capacities given; older rows are not kept).
 *   series:     [rows][slots][3] (E, Ree^2, Rg^2) after each sweep, before
 *               the exchange step;
 *   accept_log: [rows][words] bit m%64 of word m/64 of a slot's run of
 *               ceil(N/64) words = move m accepted; slots in order;
 *   exch_log:   [rows][slots] 1 accepted / 0 rejected for the lower slot of
 *               each attempted pair, 0xFF otherwise.
 * *rows receives the number of rows copied. */
PT_API int pt_get_series(pt_handle *h, double *h_series, int64_t *rows);
PT_API int pt_get_logs(pt_handle *h, uint64_t *h_accept_log, int64_t *accept_rows,
                       uint8_t *h_exch_log, int64_t *exch_rows);

/* Autotuner of the mapping.  For every distinct chain length of the batch it
 * times each mapping with 64 W B in [N, max(64, 4N)) -- with W = 1 and B <= 2
 * also packed two and four replicas per wavefront (PT_MAP_PACK2, PT_MAP_PACK4),
 * and, for PT_FP64, one lane per replica (PT_MAP_LANE) -- on the batch's chains
 * of that length
 * (their own slots, ladders, coordinates, precision and schedule) over
 * trial_sweeps sweeps after a warm-up (a candidate within 3% of the best so
 * far is timed twice more and its fastest timing kept), in a device
 * workspace of its own on
 * hip_stream, and writes the fastest code to mapping_out[n_chains] (ready for
 * config.mapping).  Unless the schedule is PT_SCHED_PER_SWEEP it then times
 * the whole batch on those choices and, for each wavefront count W, with
 * every length on its fastest mapping of that W (persistent launches of
 * different W run one after another), and keeps the fastest.  The caller's
 * state is not touched; results of a run do not depend on the mapping.
 * Synchronous.
 * Errors: as pt_init, and PT_ENOMEM when the device has no room. */
PT_API int pt_autotune(const pt_model *model, const pt_config *config, int32_t trial_sweeps,
                       void *hip_stream, int32_t *mapping_out);

/* Decision digests, [slots][2], synchronous: per slot, [0] folds every
 * accept word of the slot's sweeps (the words of pt_get_logs, in order) as
 * d = mix(d ^ word), [1] folds the outcome of every exchange attempt in
 * which the slot was the lower one as d = mix(d ^ (e << 1 | accepted)); mix
 * is the SplitMix64 finaliser (Steele, Lea, Flood 2014), d starts at 0.
 * Two runs with equal digests took the same decisions (Eqs. 5, 6) without
 * keeping the logs. */
PT_API int pt_get_digests(pt_handle *h, uint64_t *h_digests);

/* Checkpoint and resume.  pt_state_bytes gives the size of the host buffer
 * (0 and an error message for a NULL handle).  pt_get_state (synchronous)
 * writes the run counters, the slot permutation, every conformation (AoS, as
 * pt_get_coords), the running energies and bounds, the accumulators, the
 * counters and the digests; it does not hold the series or logs.
 * pt_set_state (synchronous) loads such a state into a handle made for the
 * same chains, slots and seed (the precision, schedule and capacities may
 * differ): the run then continues exactly as the saved run would have.
 * Errors: PT_ENOMEM (buffer too small), PT_EINVAL (not a state, another
 * batch, a permutation that mixes chains), PT_EDOMAIN (a broken bond),
 * PT_EHIP.  pt_set_state also clears the failed state (PT_ESTATE) left by a
 * persistent run that timed out. */
PT_API size_t pt_state_bytes(pt_handle *h);
PT_API int pt_get_state(pt_handle *h, void *h_buf, size_t bytes);
PT_API int pt_set_state(pt_handle *h, const void *h_buf, size_t bytes);

/* Test hook: a factor >= 1 by which the guard bands of PT_MIXED are widened
 * (the move band around the Metropolis threshold and, for both precisions,
 * the band of the exchange test within which the FP64-order energies are
 * recomputed; 1 by default).  A wider band sends more decisions to the FP64
 * order without changing any of them, which exercises those paths.  Applies
 * to later launches.  Errors: PT_EINVAL (NULL handle, factor < 1 or not
 * finite). */
PT_API int pt_set_guard_scale(pt_handle *h, double factor);

/* Test hook: the number of polls (each a short sleep, about 2^24 by default:
 * seconds) after which a persistent or task-flow run's wait for an exchange
 * partner or an earlier task gives up.  A small value makes every wait whose
 * partner has not arrived yet time out, which exercises the failure path
 * (PT_EHIP, then PT_ESTATE until pt_set_state) while every block still exits.
 * Applies to later launches. */
PT_API int pt_set_spin_limit(pt_handle *h, uint32_t polls);

/* Timing of the sweep kernels: runs n sweeps like pt_sweep, with HIP events
 * recorded on the handle's stream around every sweep-kernel launch (a
 * persistent launch covers all n sweeps and their exchange steps), then
 * synchronises.  *sweep_ms = summed sweep-kernel time, *total_ms = wall time
 * of the whole enqueue on the stream, *launches = sweep-kernel launches. */
PT_API int pt_time_sweeps(pt_handle *h, int64_t n_sweeps, double *sweep_ms, double *total_ms,
                          int64_t *launches);

/* Mapping of each chain (any pointer may be NULL): beads per lane (a power
 * of two <= 8) and wavefronts per replica (1, 2 or 4) -- config.mapping, or
 * by default the smallest pair with 64 * wpr * bpl >= N -- and the schedule
 * of the chain's class: 1 persistent, 2 task flow, 0 one launch per sweep.
 * [n_chains] each. */
PT_API int pt_get_mapping(pt_handle *h, int32_t *beads_per_lane, int32_t *waves_per_replica,
                          int32_t *persistent);

/* Diagnostics of the device arithmetic (used by the test suite).  op:
 *   0: IEEE sqrt      1: IEEE x/y        2: deterministic log
 *   3: FENE term of r2 = x                4: LJ term of r2 = x (FP64 order)
 *   5: FP32 LJ term of the separation (x, y, 0) as PT_MIXED scores a pair
 *      whose old separation lies on the cutoff: out[2i] = 4 eps (g(r^2) -
 *      g(rc^2)) with g the FP32 bracket (= E_mod of Eq. 1 up to rounding),
 *      out[2i+1] = the error bound the mixed path uses for that pair
 *   6: Philox block: x = counter words (4 per item, as doubles), y[0], y[1] =
 *      seed low and high 32 bits (as doubles); out[4i..4i+3] = words
 *   7: FP64 pairwise tree over each group of 64 consecutive x (the wavefront
 *      reduction of the kernels), result in every out[i] of the group
 *   8: the same in FP32 (x rounded to float first); n a multiple of 64 for 7, 8
 *   9: the FP32 pair sum of one move as PT_MIXED scores it (Eqs. 1-2, 4:
 *      sum over j != k of the new minus the old Lennard-Jones term of bead k)
 *      at 8 beads per lane and one wavefront: x holds n items of 1544
 *      doubles, 512 beads (x, y, z; beads j >= N unused), then N (2..512),
 *      k (0..N-1) and the displacement (dx, dy, dz), 3 more unused;
 *      out[2i] = the mixed sum, out[2i+1] = the rigorous bound on its error
 *      that the guard band of the Metropolis decision uses
 * Inputs and outputs are host arrays of n items; synchronous; allocates a
 * temporary device buffer. */
PT_API int pt_selftest(const pt_model *model, int op, const double *h_x, const double *h_y,
                       double *h_out, int64_t n);

/* For callers that cannot allocate device memory (code running while a HIP
 * graph is being captured around it, tight serving loops, harnesses that
 * forbid hipMalloc): pt_selftest with the same ops, arguments, results and
 * errors, whose device staging (inputs, second input, outputs) lives in a
 * fixed device array of 2^21 doubles (16 MiB) per GPU, held from the first
 * call on that GPU until the process ends, instead of buffers allocated per
 * call.  Calls no hipMalloc or hipFree.  A call needing more staging than the
 * array holds (n items need n + n + n doubles for ops 0-4, 7 and 8 -- the
 * second input only for op 1 --, 4n + 2 + 4n for op 6, 2n + 2n for op 5 and
 * 1544 n + 2 n for op 9) fails with PT_EINVAL before any device work.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (from
 * several host threads) race and must be serialised by the caller.
 * Synchronous, on the null stream of the current device. */
PT_API int pt_selftest_noalloc(const pt_model *model, int op, const double *h_x, const double *h_y,
                               double *h_out, int64_t n);

PT_API void pt_destroy(pt_handle *h);
PT_API const char *pt_last_error(void);

#endif /* PT_H */
