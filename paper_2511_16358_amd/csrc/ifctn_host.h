// Host-side job interface shared by the C ABI (ifctn_api.hip) and the serving
// runtime (ifctn_server.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "ifctn.h"

namespace ifctn {

// Tuning options of ifctn_set_option that shape a job's work plans and so
// its size.  A job is sized and created with one snapshot of them.
struct PlanOpts {
  long long phased_min, contract_div, contract_emin, contract_jmax;
  long long ugroup;   // partial slots per group of the contraction's grouped reduction (0 = off)
  bool merge_gram, onelaunch;
  int gamma;          // Gamma route: 0 never, 1 where the block would otherwise be phased, 2 wherever it fits
  bool overlap;       // Gamma route: the contraction on a second stream, concurrent with Gamma_k
};
PlanOpts current_opts();

// Fault injection for the serving tests (option "inject_admit_failures"):
// true while injected admission failures remain, consuming one.
bool take_injected_admit_failure();

// Device bytes of one job planned with these options; 0 for invalid params.
size_t job_bytes(const ifctn_params* params, const PlanOpts& opts);

// Create a job.  pool != nullptr: the job lives in [pool, pool + pool_bytes)
// (no allocation; the caller owns that memory).  check_now: synchronise and
// reject non-finite observed data at once; otherwise flag word 0 reports it.
ifctn_status job_open(const ifctn_params* params, const void* O_dev, const uint8_t* mask_dev,
                      const double* G0_host, hipStream_t stream, unsigned char* pool, size_t pool_bytes,
                      bool check_now, const PlanOpts& opts, ifctn_job** out);

hipError_t job_sweeps(ifctn_job* J, int n);       // n sweeps, X step of the last one left pending
hipError_t job_x_step(ifctn_job* J);              // the pending X step (and stop test), if any
hipError_t job_promote(ifctn_job* J);             // end the bfloat16 phase (BF16_REFINE)
bool job_is_bf16(const ifctn_job* J);
int job_refine_sweeps(const ifctn_job* J);
void job_set_stop(ifctn_job* J, double eps);      // eps > 0: device stop test after every X step
hipError_t job_reset_flags(ifctn_job* J);         // clear stop flag and sweep count
const int* job_flags(const ifctn_job* J);         // device {non-finite O, stop, sweeps counted}
hipError_t job_finalize(ifctn_job* J);            // statistics of the last sweep into job_stats_dev
const double* job_stats_dev(const ifctn_job* J);  // device double[5]
void stats_from(const double* h, int sweeps_done, ifctn_stats* out);
ifctn_status job_close(ifctn_job* J);
ifctn_status set_error(ifctn_status st, const char* msg);

}  // namespace ifctn
