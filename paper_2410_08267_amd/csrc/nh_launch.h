// Host-callable launchers of the kernels (defined next to them in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include "nh_internal.h"

namespace nh {

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s);
hipError_t launch_free_all(long long n, const TrajOut &o, hipStream_t s);
hipError_t launch_rk4_f64(const TrajParams &P, const GridPtrs &g, const TrajOut &o, const QuadAcc *qa,
                          hipStream_t s);
// qa: the fused quadrature's buffers (no per-trajectory output), or null to
// write o.ratio and o.stat for every trajectory
hipError_t launch_dp5_f64(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                          unsigned long long *counter, const QuadAcc *qa, int n_cu, hipStream_t s);
hipError_t launch_dp5_f32c(const TrajParams &P, const GridPtrs &g, const TrajOut &o,
                           unsigned long long *counter, const QuadAcc *qa, int n_cu, hipStream_t s);
// fused quadrature: scale, background sum and cleared sums before the
// trajectories; the profile after them
hipError_t launch_quad_setup(const TrajParams &P, const GridPtrs &g, const QuadAcc &qa, hipStream_t s);
// free_all: no halo (every profile point is exactly 1)
hipError_t launch_quad_finish(int n_r, const QuadAcc &qa, bool free_all, double *out, hipStream_t s);
hipError_t launch_reduce_profile(const TrajParams &P, const GridPtrs &g, const double *ratio,
                                 double *out, hipStream_t s);
hipError_t launch_reduce_stats(long long n, const TrajOut &o, unsigned long long *stats,
                               hipStream_t s);
// n_mass profiles from the same ratios: y and its weights per mass at ym, wm (mass-major)
hipError_t launch_reduce_integrand(const TrajParams &P, const GridPtrs &g, const double *ratio, double *out,
                                   hipStream_t s);
hipError_t launch_reduce_masses(const TrajParams &P, const GridPtrs &g, const double *ratio, const double *ym,
                                const double *wm, int n_mass, double *out, hipStream_t s);
// FP64 FMA throughput probe: `blocks` workgroups of 1024 threads; *flop = work of one launch
hipError_t launch_fma_probe(double *out, int blocks, hipStream_t s, double *flop);
// y[i] = f(x[i]) on the device for f = nfw_I (FN_NFW_I) or pow_factor(pw, .) (FN_POW_FACTOR)
enum { FN_NFW_I = 1, FN_POW_FACTOR = 2 };
hipError_t launch_device_fn(int fn, const PowFactor &pw, long long n, const double *x, double *y, hipStream_t s);

// slice kernels (batched and serving forms)
// nc: table columns of the launch (NCOL when any request has a moving R);
// slots: tables per workgroup (1 or 2); pow: some request of the launch has a
// power-law factor of K and Kc (PowFactor)
size_t slice_lds_bytes(bool f32c, int nc, int slots, int n_tab);
int slice_max_table_nodes(bool f32c, int nc, int slots);
hipError_t slice_capacity(bool f32c, int nc, int slots, bool pow, int n_tab, int block, int n_cu, int *grid);
hipError_t launch_slice(const SliceArgs &A, bool f32c, int nc, int slots, bool pow, int grid, int block,
                        hipStream_t s);
const void *fill_u64_kernel();
// hipFuncSetAttribute (dynamic LDS) and the occupancy query, kept per (kernel, block, bytes)
hipError_t occupancy_cached(const void *fn, int block, size_t lds, int *per_cu);
// Sets q.lds_n = n_r and grows lds by the partial sums when they fit without
// lowering per_cu (blocks per CU); q.lds_n = 0 otherwise.
hipError_t quad_lds_plan(const void *fn, int block, int per_cu, int n_r, size_t &lds, QuadAcc &q);

// A serving slice captured as a HIP graph (descriptor and order uploads, the
// in-flight clear, the slice kernel, the read-back of queue positions and
// in-flight counts), re-launched every slice with new kernel arguments.
struct SliceGraphBufs {
    void *d_desc, *d_order, *d_next, *d_inflight;          // device
    const void *h_desc, *h_order;                          // pinned host sources
    void *h_next, *h_inflight;                             // pinned host destinations
    size_t desc_bytes, order_bytes, next_bytes, inflight_bytes;
};
struct SliceGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t slice = nullptr;
    hipKernelNodeParams params{};
    SliceArgs args{};
    void *arg_ptr[1] = {nullptr};
    bool f32c = false, pow = false;
    int nc = 0, slots = 0, grid = 0, block = 0;
};
hipError_t slice_graph_build(SliceGraph &G, const SliceGraphBufs &b, const SliceArgs &A, bool f32c, int nc,
                             int slots, bool pow, int grid, int block);
hipError_t slice_graph_launch(SliceGraph &G, const SliceArgs &A, hipStream_t s);
void slice_graph_destroy(SliceGraph &G);
// profiles of the listed requests (n_blocks = their total radii; rstart[i] = first
// radius block of list[i]) and their statistics, 8 words per listed request
hipError_t launch_reduce_batch(const BatchReq *reqs, const int *list, const int *rstart, int n_list,
                               int n_blocks, unsigned long long *stats, int stat_chunks, hipStream_t s);

}  // namespace nh
