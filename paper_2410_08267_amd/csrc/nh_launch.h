// Host-callable launchers of the kernels (defined next to them in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include "nh_internal.h"

namespace nh {

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s);
hipError_t launch_free_all(long long n, const TrajOut &o, hipStream_t s);
hipError_t launch_rk4_f64(const TrajParams &P, const GridPtrs &g, const TrajOut &o, hipStream_t s);
hipError_t launch_dp5_f64(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                          unsigned long long *counter, int n_cu, hipStream_t s);
hipError_t launch_dp5_f32c(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                           unsigned long long *counter, int n_cu, hipStream_t s);
hipError_t launch_reduce_profile(const TrajParams &P, const GridPtrs &g, const double *ratio,
                                 double *out, hipStream_t s);
hipError_t launch_reduce_stats(long long n, const TrajOut &o, unsigned long long *stats,
                               hipStream_t s);
// n_mass profiles from the same ratios: y and its weights per mass at ym, wm (mass-major)
hipError_t launch_reduce_masses(const TrajParams &P, const GridPtrs &g, const double *ratio, const double *ym,
                                const double *wm, int n_mass, double *out, hipStream_t s);
// FP64 FMA throughput probe: `blocks` workgroups of 1024 threads; *flop = work of one launch
hipError_t launch_fma_probe(double *out, int blocks, hipStream_t s, double *flop);

// slice kernels (batched and serving forms)
// nc: table columns of the launch (NCOL when any request has a moving R);
// slots: tables per workgroup (1 or 2)
size_t slice_lds_bytes(bool f32c, int nc, int slots, int n_tab);
int slice_max_table_nodes(bool f32c, int nc, int slots);
hipError_t slice_capacity(bool f32c, int nc, int slots, int n_tab, int block, int n_cu, int *grid);
hipError_t launch_slice(const SliceArgs &A, bool f32c, int nc, int slots, int grid, int block, hipStream_t s);
// profiles of the listed requests (n_blocks = their total radii; rstart[i] = first
// radius block of list[i]) and their statistics, 8 words per listed request
hipError_t launch_reduce_batch(const BatchReq *reqs, const int *list, const int *rstart, int n_list,
                               int n_blocks, unsigned long long *stats, int stat_chunks, hipStream_t s);

}  // namespace nh
