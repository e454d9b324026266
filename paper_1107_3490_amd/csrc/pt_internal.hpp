// pt_internal.hpp -- structures shared by the host runtime and the kernels of
// libpt.so (replica-exchange Metropolis for a bead-spring homopolymer,
// Gross-Janke-Bachmann, arXiv:1107.3490).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

// Model constants as the kernels use them.  The FP64 ones follow the fixed
// expressions of the public header (Sec. 3.1, Eqs. 1-3); the FP32 ones are
// their round-to-nearest images for the mixed path.
struct Consts {
    double sig2, rc2, four_eps, e_rc, fene_cf, r0, R, edge;
    float sig2_f, rc2_f, four_eps_f, e_rc_f;
    // Mixed-path move bound: |S_fp32 - S_exact| <= kbound * sum_j (s6^2 + s6)
    // over both evaluations of every pair (derivation next to lj32, pt_device.hpp).
    double kbound;
    // Largest |E_mod| of an attractive pair, slightly inflated: the LJ terms
    // that are negative never go below -neg_floor (used by the energy bound).
    double neg_floor;
    // A sweep ends with an FP64-order recomputation of the running energy when
    // its bound exceeds resync_rel * max(1, |E|).
    double resync_rel;
};

// Counters per slot (see pt_observables).
constexpr int PT_NCOUNTS = 7;

// Everything a kernel needs, passed by value.
struct Tables {
    // per global slot g
    const int32_t *slot_chain;   // chain of slot g
    const int32_t *slot_index;   // position of g inside its chain
    const uint32_t *slot_gid;    // stream id of slot g (counter word 2 of its moves)
    const double *beta;          // inverse temperature of slot g
    int32_t *perm;               // conformation held by slot g
    double *acc;                 // [g][5] n, sum E, sum E^2, sum Rg^2, sum Ree^2
    int64_t *counts;             // [g][PT_NCOUNTS] see pt_observables
    const int64_t *word_off;     // accept-log word offset of slot g
    // per conformation q (conformation q starts in slot q)
    double *coords;              // swizzled SoA, bead j at (j mod B) * 64 W + j / B
    const int64_t *coord_off;    // start of conformation q in coords
    double *e_run;               // running energy
    double *b_run;               // bound on |e_run - exact sum of the FP64 terms|
    int32_t *slot_of;            // slot holding conformation q (inverse of perm)
    int64_t *done;               // persistent runs: sweeps completed by conformation q
    int64_t *dec;                // persistent runs: exchange steps decided for q's pair
    int32_t *err;                // persistent runs: nonzero after a synchronisation timeout
    uint64_t *dig;               // [S][2] digests of the accept words and exchange outcomes
    int64_t *flow_ready;         // task flow: slot g's conformation is settled for sweeps < value
    int64_t *flow_arr;           // task flow: arrivals at the pair whose lower slot is g (2 per attempt)
    int64_t *flow_task;          // task flow: next task
    // per chain c
    const int32_t *chain_n;      // beads
    const int32_t *chain_slots;  // slots
    const int32_t *chain_slot0;  // first global slot
    const uint32_t *chain_sid;   // stream chain id (exchange counters)
    const int32_t *chain_bpl;    // beads per lane of the chain's mapping
    // run state: te[0] = sweeps done (t), te[1] = exchange steps done (e)
    int64_t *te;
    // optional records
    uint64_t *accept_log;
    int64_t log_cap;
    int64_t words_total;
    uint8_t *exch_log;
    double *series;
    int64_t series_cap;
    int32_t total_slots;
    int32_t exchange_every;
    uint32_t spin_limit;         // polls of a persistent run's partner wait before it gives up
    double guard_scale;          // >= 1: widening of the guard bands (test hook; 1 by default)
    int32_t full_energy;         // nonzero: every sweep ends with the FP64-order energy
    int32_t fp64_on_accept;      // nonzero (mixed): accepted moves are re-scored in the FP64 order
    uint64_t seed;
    Consts k;
};

// Kernel launchers (pt_kernels.hip).  A class is (bpl, wpr): beads per lane
// and wavefronts per replica; list = global slots (sweep), conformations or
// slots (energy) or chains (exchange) of that class.
hipError_t launch_sweep(int bpl, int wpr, bool mixed, const Tables &T, const int32_t *slot_list,
                        int n_items, hipStream_t s);
// One lane per replica (FP64 order): same results as launch_sweep.
// One sweep and record of the slots in pack_list, `pack` (2 or 4) slots of one
// chain per wavefront (entries -1: none), chains of the (bpl, 1) layout with
// bpl = 1 or 2; n_blocks = entries / pack.
hipError_t launch_sweep_pack(int bpl, int pack, bool mixed, const Tables &T, const int32_t *pack_list,
                             int n_blocks, hipStream_t s);
hipError_t launch_sweep_lane(int bpl, int wpr, const Tables &T, const int32_t *slot_list, int n_items,
                             hipStream_t s);
hipError_t launch_energy(int bpl, int wpr, const Tables &T, const int32_t *conf_list, int n_items,
                         double *out_e, double *out_b, hipStream_t s);
// The paper's one-pair-per-thread energy of each slot's conformation (not the
// FP64 order), with a rigorous error bound; out_e / out_b indexed by slot.
hipError_t launch_energy_pairs(int bpl, int wpr, const Tables &T, const int32_t *slot_list, int n_items,
                               double *out_e, double *out_b, hipStream_t s);
hipError_t launch_exchange(int bpl, int wpr, const Tables &T, const int32_t *chain_list, int n_chains,
                           int max_pairs, int force, hipStream_t s);
hipError_t launch_advance(const Tables &T, int force, hipStream_t s);
// Persistent run of n_sweeps sweeps and exchange steps for the conformations
// in conf_list (chains of one wavefront count wpr, any bead counts per lane up
// to max_bpl).  Every block must be resident at once: the caller checks
// n_items against run_capacity first.  dense selects the build whose
// registers leave room for more blocks per compute unit.  Starts at the run
// counters in device memory.  No device query: safe inside a graph capture.
hipError_t run_capacity(int wpr, bool mixed, int max_bpl, bool dense, int64_t *blocks);
hipError_t launch_run(int wpr, bool mixed, bool dense, const Tables &T, const int32_t *conf_list,
                      int n_items, int max_bpl, int64_t n_sweeps, hipStream_t s);
// Task flow of n_sweeps sweeps and exchange steps for one class whose slots do
// not all fit on the device at once, on `resident` blocks (flow_capacity);
// starts at the run counters in device memory.
hipError_t flow_capacity(int bpl, int wpr, bool mixed, int64_t *blocks);
hipError_t launch_flow(int bpl, int wpr, bool mixed, const Tables &T, const int32_t *slot_list,
                       int n_items, int64_t n_sweeps, int64_t resident, hipStream_t s);
// Run counters past n sweeps of persistent or task-flow launches.
hipError_t launch_advance_n(const Tables &T, int64_t n, hipStream_t s);
// Diagnostics of the device arithmetic (ops of pt_selftest).  Op 9 items are
// kMoveItem doubles: 512 beads (x, y, z), then N, the moved bead k and the
// displacement (dx, dy, dz), padded.
constexpr int64_t kMoveItem = 3 * 512 + 8;
hipError_t launch_selftest(const Consts &k, int op, const double *x, const double *y,
                           double *out, int64_t n, hipStream_t s);

}  // namespace pt
