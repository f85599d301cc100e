// Entry points shared between the two translation units of libfewfit that
// are not part of its C ABI.
#pragma once

#include <cstdint>

// log of the wave efficiency of a launch of `groups` work-groups on `cus`
// compute units: groups / (ceil(groups / cus) * cus); 0 for no work-groups.
double ptune_log_wave_efficiency(int64_t groups, int cus);

// log2 of a size, sizes below 1 counted as 1 (the dispatch's shape metric).
double ptune_log2_size(int64_t x);

// The dispatch rule of ptune_dispatch on precomputed quantities: train_lg
// (nullable) the training shapes' log2 sizes (ntrain x 3), lw_train[i*k + j]
// the log wave efficiency of member j on training shape i and lw_query[j]
// at (M, N, K); lw_train == nullptr means no wave correction.
int ptune_dispatch_lw(int ntrain, const int64_t* train_mnk, const double* train_lg, int k, const int* members,
                      const double* cost, const double* lw_train, const double* lw_query, int64_t M, int64_t N,
                      int64_t K);
