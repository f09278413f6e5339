// The opaque nh_context and host helpers shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>

#include "nh_internal.h"

namespace nh {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

// Byte offsets of one request's inputs inside the staged blob.
struct Staged {
    int n_tab;
    size_t off_tab, off_tabA, off_r, off_y, off_wy, off_mu, off_smu, off_wmu, off_f0;
    int n_mass;             // multi-mass solve: scaled y grids and weights per mass
    size_t off_ym, off_wm;
    int f0_kind, f0_n;
    double f0_x0, f0_inv_dx;
    size_t bytes;
};

struct ServeState;   // serving loop (host_serve.cpp)

}  // namespace nh

struct nh_context {
    int device = 0;
    int n_cu = 0;
    char err[512] = "";
    hipStream_t stream = nullptr;                    // used by nh_solve
    nh::DevBuf blob, ratio, stat, small, out;
    nh::DevBuf quad;                                 // fused quadrature sums (QuadAcc)
    nh::DevBuf bctr;                                 // batched form: counters and statistics
    void *h_stage = nullptr;                         // pinned staging for the inputs
    unsigned long long *h_stats = nullptr;           // pinned copy of the last solve's statistics
    size_t h_stage_cap = 0;
    hipEvent_t ev_done = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
    bool pending = false;
    long long last_n_traj = -1;
    bool last_traj_kept = false;                     // the last solve stored per-trajectory results
    bool keep_traj = false;                          // NH_OPT_TRAJECTORY_STATS
    // tunables (nh_set_option)
    int queue_order = nh::ORDER_NATURAL;
    bool free_exit = true;
    double h_fp64 = 1.0e-6;                          // FP32C: |h| below this runs in FP64
    double rtol32 = 1.0e-7;                          // FP32C: tolerance floor of the FP32 attempts
    int table_nodes = 0;                             // 0: default_table_nodes()
    int block_threads = 0;                           // Dormand-Prince workgroup size (0: default)
    int batch_slots = 0;                             // tables per workgroup, batched form (0: default)
    // nh_autotune's choices per precision [FP64, FP32C] (0: built-in default)
    int tuned_plain_block[2] = {0, 0};
    int tuned_batch_block[2] = {0, 0};
    int tuned_batch_slots[2] = {0, 0};
    double slice_us = 4000.0;                        // serving: time slice length
    bool serve_graph = true;                         // serving: slices as HIP graph replays
    int max_workgroups = 0;                          // plain Dormand-Prince launches (0: one per CU)
    nh::ServeState *serve = nullptr;
};

namespace nh {

int set_err(nh_context *ctx, int code, const char *fmt, ...);
int ensure_dev(nh_context *ctx, DevBuf &b, size_t bytes);
int ensure_pinned(nh_context *ctx, size_t bytes);
Staged stage_layout(const nh_request *q, int table_nodes, int n_mass = 0);
void stage_fill(const nh_request *q, const Staged &s, char *base, TrajParams &P, int table_threads,
                const double *m_eV = nullptr);
GridPtrs grid_ptrs(const Staged &s, const char *dev);
size_t per_traj_bytes(const nh_request *q);
void serve_shutdown(nh_context *ctx);
bool serve_idle(nh_context *ctx);
int wait_pending(nh_context *ctx);
// Device buffers of one plain solve: staged inputs, the counter and statistics
// words (counter at small[0], statistics at small[8..15]), and either the
// fused quadrature's sums (qa.num != null) or per-trajectory results.
struct SolveBufs {
    char *blob;
    unsigned long long *small;
    QuadAcc qa;
    double *ratio;
    TrajStat *stat;
};
// Enqueue the kernels of one plain solve whose inputs are staged in b.blob.
int solve_launch(nh_context *ctx, const nh_request *q, const Staged &s, TrajParams P, const SolveBufs &b,
                 double *d_out, hipStream_t stream, int n_mass, double *d_integrand);
size_t quad_bytes(int n_r);
QuadAcc quad_acc(void *base, int n_r, unsigned long long *stats);
// Enqueue one plain solve: trajectories, then the profile (or one profile per
// mass), and optionally the angle-integrated distribution per radius and momentum.
int solve_enqueue(nh_context *ctx, const nh_request *q, double *d_out, double *d_ratio, hipStream_t stream,
                  int n_mass, const double *m_eV, double *d_integrand = nullptr);
int collect_stats(nh_context *ctx, nh_stats *out);
int request_columns(const nh_request *q);
int batch_slots(const nh_context *ctx, bool f32c);
int batch_block(const nh_context *ctx, bool f32c, int slots);
int batch_table_nodes(nh_context *ctx, bool f32c, int nc, int slots, int *n_tab);

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return set_err(ctx, NH_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));     \
    } while (0)

}  // namespace nh
