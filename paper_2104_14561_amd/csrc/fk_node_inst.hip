// fk_node_inst.hip -- thread-per-node and separable-box launchers for one
// (precision, dimension) pair, forward step or adjoint.
//
// The build compiles this file once per combination with
//   FK_INST_F32 = 0 | 1, FK_INST_D = 1 | 2 | 3, FK_INST_ADJ = 0 | 1
// and FK_INST_NAME set to the entry point declared in fk_internal.h
// (step_node_f32_d2, adjoint_node_f64_d3, ...), so that the heavily unrolled
// specialisations over Q* compile in parallel.  Each entry point returns
// false when the plan's Q* has no specialisation here; the caller then uses
// the lane-group kernels, which take any Q*.
//
// The separable-box kernels are compiled for d >= 2 on affine axes only: in
// one dimension the thread-per-node kernel already contracts a single axis,
// and the plan builder enables the box form only for plans whose axes are all
// affine (box_compiled).  The adjoint has its own lists (P.adj): in 2D its box
// classes are L = 4 and 6, where the saved scatter adds outweigh the cost of
// building the weight vectors.
#include "fk_device.h"

#if !defined(FK_INST_F32) || !defined(FK_INST_D) || !defined(FK_INST_ADJ) || !defined(FK_INST_NAME)
#error "fk_node_inst.hip needs FK_INST_F32, FK_INST_D, FK_INST_ADJ and FK_INST_NAME"
#endif

namespace fk {
namespace {

#if FK_INST_F32
using InstT = float;
#else
using InstT = double;
#endif
constexpr int kInstD = FK_INST_D;

#if !FK_INST_ADJ

template <typename T, int D, int QS>
void step_node_launch(const PlanDev &P, int n, const void *packed, void *u_out, hipStream_t s)
{
    constexpr int GS = (QS <= 2) ? 2 : (QS <= 4) ? 4 : (QS <= 8) ? 8 : 16;
    // TW: the R2 interpolant, whose records carry the twist field; FC: face
    // kinds other than exit-1 or node-dependent diffusion (never with R2: the
    // plan builder sends those plans to the lane-group step)
#define FK_NODE_TW(G_, AFF_, TW_, FC_, grid_, nw_, wl_)                                        \
    k_step_node<T, D, QS, G_, AFF_, TW_, FC_><<<grid_, kBlock, 0, s>>>(                        \
        P, n, nw_, P.inst, wl_, P.fw_nodes, P.trig, P.coords, (const T *)packed, (T *)u_out)
#define FK_NODE(G_, AFF_, grid_, nw_, wl_)                                                     \
    do {                                                                                       \
        if (P.faces) { FK_NODE_TW(G_, AFF_, false, true, grid_, nw_, wl_); break; }            \
        if constexpr (D >= 2) {                                                                \
            if (P.hermite2) { FK_NODE_TW(G_, AFF_, true, false, grid_, nw_, wl_); break; }     \
        }                                                                                      \
        FK_NODE_TW(G_, AFF_, false, false, grid_, nw_, wl_);                                   \
    } while (0)
    if (P.n_fw_work > 0) {
        if (P.step_kind == 2) {
            if (P.all_affine) FK_NODE(GS, true, P.fw_split_grid, P.n_fw_split_work, P.fw_split_work);
            else FK_NODE(GS, false, P.fw_split_grid, P.n_fw_split_work, P.fw_split_work);
        } else {
            if (P.all_affine) FK_NODE(1, true, P.fw_grid, P.n_fw_work, P.fw_work);
            else FK_NODE(1, false, P.fw_grid, P.n_fw_work, P.fw_work);
        }
    }
#undef FK_NODE
#undef FK_NODE_TW
    if constexpr (D >= 2) {
        // separable nodes, one launch per footprint class
#define FK_BOX(c_, L_)                                                                         \
        if (P.n_box_work[c_] > 0)                                                              \
            k_step_box<T, D, QS, L_, true><<<P.box_grid[c_], kBlock, 0, s>>>(                  \
                P, n, P.n_box_work[c_], P.inst, P.box_work + P.box_work_off[c_], P.box_nodes,  \
                P.trig, P.coords, (const T *)packed, (T *)u_out);
        FK_BOX(0, 3) FK_BOX(1, 4) FK_BOX(2, 5) FK_BOX(3, 6) FK_BOX(4, 8)
#undef FK_BOX
    }
}

#else

template <typename T, int D, int QS>
void adjoint_node_launch(const PlanDev &P, int n, const void *packed, const void *lam, void *mu,
                         double *grad, hipStream_t s)
{
    const size_t lds = (size_t)P.tile_elems * sizeof(double);   // FP64 tiles
    const AdjLists &A = P.adj;
    // interior items (no exit tests; 2D plans only) first, then the rest
    if constexpr (D == 2) if (A.n_in_work > 0) {
        if (P.all_affine)
            k_adjoint_node<T, D, QS, true, true><<<A.in_grid, kBlock, lds, s>>>(
                P, n, A.n_in_work, P.inst, A.fw_work, A.fw_tiles, A.fw_nodes, P.trig, P.coords,
                (const T *)packed, (const T *)lam, (T *)mu, grad);
        else
            k_adjoint_node<T, D, QS, false, true><<<A.in_grid, kBlock, lds, s>>>(
                P, n, A.n_in_work, P.inst, A.fw_work, A.fw_tiles, A.fw_nodes, P.trig, P.coords,
                (const T *)packed, (const T *)lam, (T *)mu, grad);
    }
    if (A.n_fw_work > 0) {
        const WorkItem *wk = A.fw_work + A.n_in_work;
        const TileBox *tl = A.fw_tiles + A.n_in_work;
        if (P.all_affine)
            k_adjoint_node<T, D, QS, true, false><<<A.fw_grid, kBlock, lds, s>>>(
                P, n, A.n_fw_work, P.inst, wk, tl, A.fw_nodes, P.trig, P.coords,
                (const T *)packed, (const T *)lam, (T *)mu, grad);
        else
            k_adjoint_node<T, D, QS, false, false><<<A.fw_grid, kBlock, lds, s>>>(
                P, n, A.n_fw_work, P.inst, wk, tl, A.fw_nodes, P.trig, P.coords,
                (const T *)packed, (const T *)lam, (T *)mu, grad);
    }
    if constexpr (D == 2) {
#define FK_ABOX(c_, L_)                                                                        \
        if (A.n_box_work[c_] > 0)                                                              \
            k_adjoint_box2<T, QS, L_><<<A.box_grid[c_], kBlock, lds, s>>>(                     \
                P, n, A.n_box_work[c_], P.inst, A.box_work + A.box_work_off[c_],               \
                A.box_tiles + A.box_work_off[c_], A.box_nodes, P.trig, P.coords,               \
                (const T *)packed, (const T *)lam, (T *)mu, grad);
        FK_ABOX(0, 4) FK_ABOX(1, 6)
#undef FK_ABOX
    } else if constexpr (D == 3) {
#define FK_ABOX(c_, L_)                                                                        \
        if (A.n_box_work[c_] > 0)                                                              \
            k_adjoint_box<T, D, QS, L_, true><<<A.box_grid[c_], kBlock, lds, s>>>(             \
                P, n, A.n_box_work[c_], P.inst, A.box_work + A.box_work_off[c_],               \
                A.box_tiles + A.box_work_off[c_], A.box_nodes, P.trig, P.coords,               \
                (const T *)packed, (const T *)lam, (T *)mu, grad);
        FK_ABOX(0, 3) FK_ABOX(1, 4) FK_ABOX(2, 5) FK_ABOX(3, 6) FK_ABOX(4, 8)
#undef FK_ABOX
    }
}

#endif

}  // namespace

#if !FK_INST_ADJ
bool FK_INST_NAME(const PlanDev &P, int n, const void *packed, void *u_out, hipStream_t s)
{
    if (P.d != kInstD) return false;
    bool any_box = false;
    for (int c = 0; c < kBoxClasses; ++c) any_box = any_box || P.n_box_work[c] > 0;
    if (any_box && !(kInstD >= 2 && P.all_affine)) return false;
#define FK_QS(v) case v: step_node_launch<InstT, kInstD, v>(P, n, packed, u_out, s); return true;
#else
bool FK_INST_NAME(const PlanDev &P, int n, const void *packed, const void *lam, void *mu,
                  double *grad, hipStream_t s)
{
    if (P.d != kInstD) return false;
    bool any_box = false;
    for (int c = 0; c < kBoxClasses; ++c) any_box = any_box || P.adj.n_box_work[c] > 0;
    if (any_box && !(kInstD >= 2 && P.all_affine)) return false;
#define FK_QS(v) case v: adjoint_node_launch<InstT, kInstD, v>(P, n, packed, lam, mu, grad, s); return true;
#endif
#if FK_INST_D == 1
    switch (P.qs) { FK_QS(2) FK_QS(3) FK_QS(4) FK_QS(5) FK_QS(6) FK_QS(7) FK_QS(8)
                    FK_QS(10) FK_QS(12) FK_QS(16) default: return false; }
#elif FK_INST_D == 2
    switch (P.qs) { FK_QS(2) FK_QS(3) FK_QS(4) FK_QS(5) FK_QS(6) FK_QS(7) FK_QS(8)
                    default: return false; }
#else
    switch (P.qs) { FK_QS(2) FK_QS(3) FK_QS(4) FK_QS(5) FK_QS(6) default: return false; }
#endif
#undef FK_QS
}

}  // namespace fk
