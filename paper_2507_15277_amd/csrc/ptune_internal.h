// Entry points shared between the two translation units of libfewfit that
// are not part of its C ABI.
#pragma once

#include <cstdint>

// log of the wave efficiency of a launch of `groups` work-groups on `cus`
// compute units: groups / (ceil(groups / cus) * cus); 0 for no work-groups.
double ptune_log_wave_efficiency(int64_t groups, int cus);

// The dispatch rule of ptune_dispatch on precomputed log wave efficiencies:
// lw_train[i*k + j] for member j on training shape i and lw_query[j] at
// (M, N, K); lw_train == nullptr means no wave correction.
int ptune_dispatch_lw(int ntrain, const int64_t* train_mnk, int k, const int* members, const double* cost,
                      const double* lw_train, const double* lw_query, int64_t M, int64_t N, int64_t K);
