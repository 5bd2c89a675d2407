// Host-side pieces of the solve launchers shared between translation units.
#pragma once
#include "radiotrace_mlp.h"
#include "radiotrace_solve.h"

namespace rt {

// Enqueue a solve of up to n_cap pairs (the number read on the device from
// *n_dev when n_dev is not NULL); arguments already validated; the workspace
// is rt_solve_workspace_bytes(field, n_cap, prm) bytes.  fam_mask (device,
// per pair, may be NULL): bit f set = solve family f; the entries of the
// other family are reported as no solution.
rt_status solve_enqueue(const rt_field* field, const rt_boundaries* bnd, double tol,
                        const rt_step_limits* L, const rt_pairs* pairs, int64_t n_cap,
                        const int64_t* n_dev, const uint8_t* fam_mask,
                        const rt_solve_params* prm, const rt_solve_outputs* out, void* workspace,
                        void* stream, const rt_tuning* tuning);

// Enqueue the seeded secant of the entries [2 n] with seed_try set; the
// workspace needs 4 KiB.
rt_status seeded_enqueue(const rt_field* field, const rt_boundaries* bnd, double tol,
                         const rt_step_limits* L, const rt_pairs* pairs, const double* seed,
                         const int32_t* seed_try, const rt_surrogate_params* sp,
                         const rt_solve_outputs* out, int32_t* verify, void* workspace,
                         void* stream, const rt_tuning* tuning);

rt_status check_surrogate_params(const rt_surrogate_params* sp);

}  // namespace rt
