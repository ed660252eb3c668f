// Peak probes (probe.hip): the vector-ALU rates the device sustains.
#pragma once

#include <cstdint>

namespace envpot {

// Times in ms of independent v_fma_f32, v_fma_f64 and v_rsq_f32 streams
// (ms_out[0..2]); returns 0 on success.
int run_peak_probe(double* ms_out);

// Lane operations each probe kernel performs.
int64_t peak_probe_lane_ops();

}  // namespace envpot
