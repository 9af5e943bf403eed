// psl_launch.h -- host-side launchers of the libpsl kernels (internal).
#pragma once

#include "psl_device.h"

namespace psl {

hipError_t launch_power_table(double *T, uint32_t n, uint32_t alpha, hipStream_t s);
hipError_t launch_init_bits(WalkDev *walks, const BatchEntry *batch, const uint32_t *want,
                            uint32_t nb, uint32_t max_nw, hipStream_t s);
hipError_t launch_corr(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint32_t max_L,
                       int only_pending, hipStream_t s);
constexpr uint32_t kPendUnit = 1024;   // shifts per work unit of the pending-walk rebuild

// After the step's C update and bookkeeping: C, F and PSL of the walks on the
// pending list (pend: count, then batch positions) that switched phase, in
// work units of kPendUnit shifts (units: how many the batch's nb walks hold in
// all).
hipError_t launch_pending(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint64_t units,
                          const Tables &tabs, const uint32_t *pend, hipStream_t s);
hipError_t launch_fitness(WalkDev *walks, const BatchEntry *batch, uint32_t nb, const Tables &tabs,
                          int mode, hipStream_t s);
hipError_t launch_eval(const WalkDev *walks, const BatchEntry *batch, const EvalItem *items,
                       uint32_t n_items, const Tables &tabs, const EvalShape &shape,
                       EvalQueues *queues, hipStream_t s);
// mode 0: the step's chunk arrays and near-peak list (and, with pend, the
// step's pending list emptied), turned into suffix values when scan != 0 (the
// evaluation in 16-wavefront blocks reads those; smaller blocks add the chunk
// values themselves); mode 2: the initial fitness (value_local, F_pivot,
// psl_pivot, psl_best) of every walk.
hipError_t launch_suffix(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint32_t max_L,
                         const Tables &tabs, int mode, const SegMap *map, uint32_t *pend, int scan,
                         hipStream_t s);
// Zero the near-peak counts of a batch, its pending count and its combine
// counters (done, nb entries; may be null) after its scratch is allocated.
hipError_t launch_near_reset(const BatchEntry *batch, uint32_t nb, uint32_t *pend, uint32_t *done, hipStream_t s);
// F and PSL per candidate from the partials, then the selection, its
// ambiguity flags (margin: their relative margin) and, pure == 0, the step's
// bookkeeping (pend: the pending list the walks that switch phase join), by
// each walk's last combine block in launches of at most 256 combine blocks
// (done: one zeroed counter per batch position, left zero; without it the
// selection takes a launch of its own): pure != 0 writes the choice record
// `out` (one walk), else the walks' step records.
hipError_t launch_select(WalkDev *walks, const BatchEntry *batch, uint32_t nb, uint32_t comb_blocks,
                         uint32_t comb_group, const Tables &tabs, int pure, void *out, uint32_t *pend,
                         uint32_t *done, double margin, hipStream_t s);
size_t choice_dev_size();
void choice_dev_unpack(const void *p, uint32_t *i_best, uint32_t *j_best, double *F_best,
                       double *F_min, uint32_t *j_psl, int32_t *psl_min, int32_t *psl_k, uint32_t *flags);
// The C update of each walk's recorded move (j_fixed < 0, after the
// bookkeeping) or of a forced flip of element j_fixed (before its bit flips).
hipError_t launch_apply(WalkDev *walks, const BatchEntry *batch, const SegMap &map, int64_t j_fixed,
                        hipStream_t s);
hipError_t launch_flip_bit(WalkDev *walks, const BatchEntry *batch, uint32_t j, hipStream_t s);
// Units of launch_pending for walks of length L.
inline uint64_t pending_units(uint32_t L) { return (L - 1 + kPendUnit - 1) / kPendUnit; }

// Split evaluation (psl_split.hip): the step's coefficients, digits, prefix
// sums, scale and path choice of the batch's split walks (after the suffix
// pass, before the evaluation), and the matrix-core linear sums (items:
// walk, 512-element block, k-split).
hipError_t launch_split_prep(const WalkDev *walks, const BatchEntry *batch, uint32_t nb, const Tables &tabs,
                             const SegMap &map, hipStream_t s);
hipError_t launch_lin(const WalkDev *walks, const BatchEntry *batch, const EvalItem *items, uint32_t n_items,
                      hipStream_t s);

}  // namespace psl
