// fk_internal.h -- device-side plan records and kernel launchers shared by the
// host runtime (fk_host.cpp) and the gfx950 kernels (fk_device.h, instantiated
// by fk_launch.hip and fk_node_inst.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fk {

constexpr int kMaxDim = 3;
constexpr int kTimeFactors = 4;   // per (step, instance) time table entries
constexpr int kThetaSlots = 8;    // gradient entries per instance (FK_MAX_THETA)
constexpr int kBoxClasses = 5;    // separable-form box sizes L = 3, 4, 5, 6, 8

// Per-instance record read by every kernel (one per instance of a plan).
struct DevInst {
    int d;
    int n[kMaxDim];
    int periodic[kMaxDim];
    int uniform[kMaxDim];          // nearly equal spacing: guess the cell arithmetically
    int affine[kMaxDim];           // x_k == k * step + lo exactly (k < n-1), x_{n-1} == hi
    int coef_kind;
    int region_kind;
    int n_act;
    int pad0;
    long long stride[kMaxDim];     // node strides inside the instance
    long long node_off;            // offset of the instance in a packed field
    long long coord_off[kMaxDim];  // offsets of the axes in the coordinate array
    long long act_off;             // offset in the packed active list
    double lo[kMaxDim], hi[kMaxDim], inv_h[kMaxDim], period[kMaxDim], step[kMaxDim];
    double coef[16];
    double D;
    double center[kMaxDim];
    double r2;
    double S;       // sqrt(2 D) * sqrt(2 dt)
    double dSdD;    // S / (2 D)  (adjoint)
    // assembled (ELL) form: this instance's row box, width (box nodes x
    // (d + 1) fields), box nodes per field padded to whole 16-byte blocks,
    // and storage offset
    int ell_box[kMaxDim];
    int ell_w;
    int ell_nbp;
    long long ell_off;
    // offset of the instance in the caller's fields: node_off, except in the
    // FP64 sub-plan of an FP32 plan, whose inputs and outputs use the
    // parent's layout
    long long out_off;
    int face[kMaxDim][2];          // FK_FACE_* per axis and side
    int sdiff;                     // diffusion depends on the node (runaway model)
    int pad1;
};

// A contiguous chunk of one instance's nodes (slope pass) or active nodes
// (step pass) handled by one workgroup.  kind 0: nodes first .. first+count-1;
// kind 1 + a: entries of the trig table of axis a.
constexpr int kEllClasses = 8;   // ELL assembly width classes

struct WorkItem {
    int inst;
    int first;
    int count;
    int kind;
};

// LDS tile of an adjoint work item: node box lo[a] .. lo[a] + ext[a] - 1.
struct TileBox {
    int lo[kMaxDim];
    int ext[kMaxDim];
    int use_lds;
    int pad;
    int soff;   // first entry of the tile's staging slot, or -1 (flush with atomics)
};

// The adjoint's work lists: active nodes handled per landing point (fw) and
// separable nodes handled in box form by footprint class, each work item with
// its LDS tile.  Box classes: L = 4, 6 in 2D; 3, 4, 5, 6, 8 in 3D.
struct AdjLists {
    const int *fw_nodes;
    const WorkItem *fw_work;
    const TileBox *fw_tiles;
    int n_fw_work;
    int fw_grid;
    // the first n_in_work items: no landing point of any of their nodes can exit
    int n_in_work;
    int in_grid;
    // tile staging: each tile's entries (fields interleaved) at its soff; per
    // node the staging entries (field 0) of the tiles that cover it
    void *stage;                // T, or null when the tiles flush with atomics
    int n_cov;                  // nodes covered by a staged tile
    const int *cov_node;        // [n_cov] packed node index
    const int *cov_ptr;         // [n_cov + 1] into cov_base
    const int *cov_base;        // staging index of field 0, per (node, covering tile)
    const int *box_nodes;
    const WorkItem *box_work;
    const TileBox *box_tiles;
    int box_work_off[kBoxClasses];
    int n_box_work[kBoxClasses];
    int box_grid[kBoxClasses];
};

// Pointers into the workspace that every launch needs.
struct PlanDev {
    const DevInst *inst;
    const double *coords;       // packed node coordinates of all axes
    const int *active;          // node index inside its instance, per active node
    const unsigned char *chi;   // terminal values (0/1) per packed node
    const double *gh_a;         // 1D GH nodes (Q*)
    const double *gh_w;         // tensor weights (Q), double
    const float *gh_wf;         // tensor weights (Q), float
    const double *gh_w1;        // 1D weights (Q*), double
    const float *gh_w1f;        // 1D weights (Q*), float
    const double *tfac;         // [n_steps][n_inst][kTimeFactors]
    double2 *trig;              // per-axis (sin, cos) of the drift arguments at t_n
    const WorkItem *slope_work; // trig table items, then node runs near active nodes
    const WorkItem *node_work;  // all nodes (adjoint passes)
    const WorkItem *act_work;   // step pass work list (block / G active nodes each)
    const WorkItem *row_work;   // row-per-thread work list (block active nodes each)
    int *flags;                 // bit 0: non-finite value produced
    int n_inst;
    int n_slope_work;
    int n_table_work;
    int n_node_work;
    int n_act_work;
    int n_row_work;
    int d;
    int qs;                     // Q*
    int n_quad;                 // Q
    int n_steps;
    int block;                  // threads per workgroup
    int group;                  // lanes per active node in the step passes
    int step_kind;              // 0: thread per node, 1: lane group, 2: split node
    int all_affine;             // every axis of every instance is affine
    int hermite2;               // R2 interpolant: 2D twist field in the records' fourth entry,
                                // 3D twist fields in a second record per node (packed2)
    void *packed2;              // 3D R2: (t01, t02, t12, t012) per node, or null
    int faces;                  // face kinds other than exit-1, or node-dependent diffusion
    // forward step work: nodes handled per landing point (fw) and separable
    // nodes handled in box form, by box class
    const int *fw_nodes;
    const WorkItem *fw_work;
    int n_fw_work;
    int fw_grid;
    const WorkItem *fw_split_work;
    int n_fw_split_work;
    int fw_split_grid;
    const int *box_nodes;
    const WorkItem *box_work;
    int box_work_off[kBoxClasses];
    int n_box_work[kBoxClasses];
    int box_grid[kBoxClasses];
    AdjLists adj;               // adjoint step work
    int tile_elems;             // LDS entries (FP64) of the largest adjoint tile in use
    const WorkItem *split_work; // chunks of block / pow2(Q*) active nodes
    int n_split_work;
    int split_grid;
    int slope_grid;             // workgroups of the slope pass
    int node_grid;              // workgroups of all-node passes
    int act_grid;               // workgroups of the step pass
    int row_grid;               // workgroups of row-per-thread passes
    double dt;
    double t0;
    long long n_nodes;
    long long n_active;
    // ELL form
    int ell_width;
    int ell_box[kMaxDim];
    int ell_grid;
    // assembly work by row-width class: the LDS row boxes of a launch are
    // sized by its class's widest row, not by the widest row of the plan
    const WorkItem *ell_work;
    const WorkItem *ell_sep_work;   // separable rows, assembled as outer products,
    int n_ell_sep_cls;              // by class of the longest box axis
    int ell_sep_off[kEllClasses];
    int ell_sep_n[kEllClasses];
    int ell_sep_l[kEllClasses];     // longest box axis in the class (LDS vectors)
    int ell_sep_tb[kEllClasses];    // bytes of the class's largest block table
    int ell_sep_grid[kEllClasses];
    int n_ell_cls;
    int ell_cls_off[kEllClasses];
    int ell_cls_n[kEllClasses];
    int ell_cls_w[kEllClasses];
    int ell_cls_grid[kEllClasses];
};

// Kernel launchers (fk_launch.hip).  T is double or float; all return the
// HIP error of the launch.
hipError_t launch_init_field(const PlanDev &P, bool f32, void *u, hipStream_t s);
hipError_t launch_slopes(const PlanDev &P, bool f32, int n, const void *u, void *packed,
                         hipStream_t s);
hipError_t launch_tables(const PlanDev &P, int n, hipStream_t s);
hipError_t launch_step_fused(const PlanDev &P, bool f32, int n, const void *packed,
                             void *u_out, hipStream_t s);
bool step_node_compiled(int d, int qs);
// LDS bytes of a separable-assembly launch: the axis vectors of 64 rows
// (d x 2 x lm columns) and a zero column, then the class's block table
inline size_t ell_sep_lds(int d, int lm, int tb, bool f32)
{
    return (size_t)(d * 2 * lm + 1) * 64 * (f32 ? 4 : 8) + (size_t)tb;
}
// Workgroups of an assembly kernel resident per CU at an LDS size, at most 8
// (the persistent grids of the assembly are sized so that every workgroup is
// resident at once): sep = the separable kernel (256 threads), else the
// LDS-box kernel with lane groups of G.  *out = 8 when the query fails.
hipError_t ell_per_cu(int d, int G, bool f32, bool sep, size_t lds, int *out);
// the separable-box form: d >= 2, affine axes, a compiled Q*
bool box_compiled(int d, int qs);

// Thread-per-node and separable-box launchers, one per (precision, dimension)
// (fk_node_inst.hip).  Each returns false when the plan's Q* (or its mix of
// box work and axis kinds) has no compiled specialisation.
#define FK_NODE_ENTRY(name) \
    bool name(const PlanDev &P, int n, const void *packed, void *u_out, hipStream_t s);
#define FK_ADJ_ENTRY(name)                                                                  \
    bool name(const PlanDev &P, int n, const void *packed, const void *lam, void *mu,       \
              double *grad, hipStream_t s);
FK_NODE_ENTRY(step_node_f32_d1) FK_NODE_ENTRY(step_node_f32_d2) FK_NODE_ENTRY(step_node_f32_d3)
FK_NODE_ENTRY(step_node_f64_d1) FK_NODE_ENTRY(step_node_f64_d2) FK_NODE_ENTRY(step_node_f64_d3)
FK_ADJ_ENTRY(adjoint_node_f32_d1) FK_ADJ_ENTRY(adjoint_node_f32_d2) FK_ADJ_ENTRY(adjoint_node_f32_d3)
FK_ADJ_ENTRY(adjoint_node_f64_d1) FK_ADJ_ENTRY(adjoint_node_f64_d2) FK_ADJ_ENTRY(adjoint_node_f64_d3)
#undef FK_NODE_ENTRY
#undef FK_ADJ_ENTRY
hipError_t launch_assemble_ell(const PlanDev &P, bool f32, int n, int *org, void *vals,
                               void *exit_mass, hipStream_t s);
hipError_t launch_ell_apply(const PlanDev &P, bool f32, const int *org, const void *vals,
                            const void *exit_mass, const void *packed, void *u_out,
                            hipStream_t s);
// The assembled operator applied to nc <= 4 columns (records of column c at
// packed + c * plane elements, its field at u_out + c * fstride elements).
hipError_t launch_ell_apply_mc(const PlanDev &P, bool f32, const int *org, const void *vals,
                               const void *exit_mass, const void *packed, long long plane,
                               void *u_out, long long fstride, int nc, hipStream_t s);
hipError_t launch_export_ell(const PlanDev &P, bool f32, const int *org_in, const void *vals_in,
                             int *cols_out, void *vals_out, hipStream_t s);
hipError_t launch_export_cells(const PlanDev &P, int inst, int n, int *cells,
                               unsigned char *exit_flags, hipStream_t s);
hipError_t launch_clear_flags(const PlanDev &P, hipStream_t s);

// Adjoint launchers.
// part 0: the whole transposed step; 1: the per-point work list only (or the
// lane-group form); 2: the separable-box lists only
hipError_t launch_adjoint_step(const PlanDev &P, bool f32, int n, const void *packed,
                               const void *lam, void *mu, double *grad, hipStream_t s,
                               int part = 0);
hipError_t launch_adjoint_slopes_T(const PlanDev &P, bool f32, const void *u, void *mu,
                                   void *lam_next, hipStream_t s);
hipError_t launch_adjoint_init(const PlanDev &P, bool f32, const void *lam0, void *lam,
                               hipStream_t s, bool lam0_parent_f32 = false);
// FP64 sub-plan <-> the parent FP32 plan's fields: out[out_off + j] =
// (float) u[node_off + j] and back, over every node of every instance.
hipError_t launch_convert_out(const PlanDev &P, const double *u, float *out, hipStream_t s);
hipError_t launch_convert_in(const PlanDev &P, const float *in, double *u, hipStream_t s);
// out[inst] = max over the instance's nodes of |a - b| (out cleared by the caller)
hipError_t launch_inst_maxdiff(const PlanDev &P, const double *a, const float *b, double *out,
                               hipStream_t s);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// LDS atomic throughput probe (measurement): blocks x 256 lanes, iters
// conflict-free ds_add per lane, out[blocks] written.
hipError_t launch_lds_atomic_probe(bool f32, int blocks, int iters, double *out, hipStream_t s);

// Device address of the static scratch array on the current device (taken
// with hipGetSymbolAddress on the first call per device).
hipError_t static_scratch(void **out);

// Step-operator hooks: (d + 1) fields <-> node records; a - b on active nodes
// and 0 elsewhere (b may be null).
hipError_t launch_pack_fields(const PlanDev &P, bool f32, const void *x, void *packed,
                              hipStream_t s);
hipError_t launch_unpack_fields(const PlanDev &P, bool f32, const void *packed, void *x,
                                hipStream_t s);
hipError_t launch_masked_diff(const PlanDev &P, bool f32, const void *a, const void *b, void *out,
                              hipStream_t s);

}  // namespace fk
