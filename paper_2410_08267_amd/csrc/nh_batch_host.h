// Host helpers shared by the batched solve and the serving loop.
#pragma once

#include <functional>

#include "nh_context.h"

namespace nh {

// Fill request q's staged inputs at host_base (layout s) and its descriptor,
// whose device pointers refer to the same layout at dev_base.
void describe(const nh_context *ctx, const nh_request *q, const Staged &s, char *host_base, const char *dev_base,
              double *ratio, TrajStat *stat, double *out, BatchReq &d);
// Validation for the batched and serving forms; precision < 0 accepts either.
int check_batchable(nh_context *ctx, const nh_request *q, int index, int precision);
// nh_stats from the 8 statistics words of one request.
void stats_from_words(const unsigned long long *w, long long n_traj, double kernel_ms, nh_stats &st);
// fn(0..n-1) on up to 16 host threads.
void parallel_for(int n, const std::function<void(int)> &fn);

}  // namespace nh
