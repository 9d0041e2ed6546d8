// fk_launch.hip -- launchers of the slope pass, the lane-group step and
// adjoint (any Q*), the assembled (ELL) form, exports and utility fills.  The
// thread-per-node and separable-box launchers live in the fk_node_inst.hip
// instances; launch_step_fused and launch_adjoint_step pick one of them when
// the plan's Q* has a compiled specialisation and fall back to the lane-group
// kernels otherwise.
#include "fk_device.h"
#include "fkexit.h"

#include <mutex>

namespace fk {

// ---------------------------------------------------------------------------
// Fixed device buffer of the allocation-free forward pass (fk_forward_static):
// one copy per device, held until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[FK_STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_init_field(const PlanDev &P, bool f32, void *u, hipStream_t s)
{
    if (f32)
        k_init_field<float><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.chi, P.n_nodes, (float *)u);
    else
        k_init_field<double><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.chi, P.n_nodes, (double *)u);
    return hipGetLastError();
}

hipError_t launch_slopes(const PlanDev &P, bool f32, int n, const void *u, void *packed,
                         hipStream_t s)
{
    FK_DISPATCH_D(P.d,
        if (f32) k_slopes<float, D><<<P.slope_grid, kBlock, 0, s>>>(P, n, 0, P.n_slope_work, (const float *)u, (float *)packed);
        else k_slopes<double, D><<<P.slope_grid, kBlock, 0, s>>>(P, n, 0, P.n_slope_work, (const double *)u, (double *)packed));
    return hipGetLastError();
}

hipError_t launch_tables(const PlanDev &P, int n, hipStream_t s)
{
    if (P.n_table_work == 0) return hipSuccess;
    const int g = P.n_table_work >= 8 ? (P.n_table_work + 7) / 8 * 8 : P.n_table_work;
    FK_DISPATCH_D(P.d,
        k_slopes<double, D><<<g, kBlock, 0, s>>>(P, n, 0, P.n_table_work, nullptr, nullptr));
    return hipGetLastError();
}

template <typename T, int D, int G, int NQ>
static void step_fused_launch(const PlanDev &P, int n, const void *packed, void *u_out,
                              hipStream_t s)
{
    k_step_fused<T, D, G, NQ><<<P.act_grid, kBlock, 0, s>>>(
        P, n, P.inst, P.act_work, P.active, P.trig, P.coords, (const T *)packed, (T *)u_out);
}

template <typename T, int D>
static hipError_t step_fused_dispatch(const PlanDev &P, int n, const void *packed, void *u_out,
                                      hipStream_t s)
{
    const int nq = (P.n_quad + P.group - 1) / P.group;
    switch (P.group) {
    case 4: step_fused_launch<T, D, 4, 1>(P, n, packed, u_out, s); break;
    case 8: step_fused_launch<T, D, 8, 1>(P, n, packed, u_out, s); break;
    case 16: step_fused_launch<T, D, 16, 1>(P, n, packed, u_out, s); break;
    case 32: step_fused_launch<T, D, 32, 1>(P, n, packed, u_out, s); break;
    case 64:
        if (nq <= 1) step_fused_launch<T, D, 64, 1>(P, n, packed, u_out, s);
        else if (nq <= 2) step_fused_launch<T, D, 64, 2>(P, n, packed, u_out, s);
        else if (nq <= 4) step_fused_launch<T, D, 64, 4>(P, n, packed, u_out, s);
        else return hipErrorInvalidValue;
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

bool step_node_compiled(int d, int qs)
{
    if (d == 1) return (qs >= 2 && qs <= 8) || qs == 10 || qs == 12 || qs == 16;
    if (d == 2) return qs >= 2 && qs <= 8;
    if (d == 3) return qs >= 2 && qs <= 6;
    return false;
}

bool box_compiled(int d, int qs)
{
    return d >= 2 && step_node_compiled(d, qs);
}

hipError_t launch_step_fused(const PlanDev &P, bool f32, int n, const void *packed, void *u_out,
                             hipStream_t s)
{
    if (P.step_kind != 1) {
        bool ok = false;
        switch (P.d) {
        case 1: ok = f32 ? step_node_f32_d1(P, n, packed, u_out, s) : step_node_f64_d1(P, n, packed, u_out, s); break;
        case 2: ok = f32 ? step_node_f32_d2(P, n, packed, u_out, s) : step_node_f64_d2(P, n, packed, u_out, s); break;
        case 3: ok = f32 ? step_node_f32_d3(P, n, packed, u_out, s) : step_node_f64_d3(P, n, packed, u_out, s); break;
        default: return hipErrorInvalidValue;
        }
        if (ok) return hipGetLastError();
    }
    FK_DISPATCH_D(P.d,
        return f32 ? step_fused_dispatch<float, D>(P, n, packed, u_out, s)
                   : step_fused_dispatch<double, D>(P, n, packed, u_out, s));
    return hipSuccess;
}

hipError_t ell_per_cu(int d, int G_, bool f32, bool sep, size_t lds, int *out)
{
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    *out = 8;
    if (sep) {
        FK_DISPATCH_D(d,
            if (f32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_assemble_ell_sep<float, D>, 256, lds);
            else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_assemble_ell_sep<double, D>, 256, lds));
    } else {
        FK_DISPATCH_D(d, FK_DISPATCH_G(G_,
            if (f32) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_assemble_ell<float, D, G>, kBlock, lds);
            else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_assemble_ell<double, D, G>, kBlock, lds)));
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();   // a failed query must not surface at a later launch check
        return e;
    }
    if (nb >= 1 && nb < 8) *out = nb;
    return hipSuccess;
}

hipError_t launch_assemble_ell(const PlanDev &P, bool f32, int n, int *org, void *vals,
                               void *exit_mass, hipStream_t s)
{
    // separable rows: direct outer-product assembly, one thread per row, one
    // launch per class of the longest box axis (LDS vectors sized by the class)
    for (int c = 0; c < P.n_ell_sep_cls; ++c) {
        const WorkItem *work = P.ell_sep_work + P.ell_sep_off[c];
        const int nw = P.ell_sep_n[c], lm = P.ell_sep_l[c], grid = P.ell_sep_grid[c];
        const size_t lds = ell_sep_lds(P.d, lm, P.ell_sep_tb[c], f32);
        FK_DISPATCH_D(P.d,
            if (f32) k_assemble_ell_sep<float, D><<<grid, 256, lds, s>>>(P, n, work, nw, lm, org, (float *)vals, (float *)exit_mass);
            else k_assemble_ell_sep<double, D><<<grid, 256, lds, s>>>(P, n, work, nw, lm, org, (double *)vals, (double *)exit_mass));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // the other rows: one launch per row-width class, its FP64 row boxes sized by the class
    for (int c = 0; c < P.n_ell_cls; ++c) {
        const WorkItem *work = P.ell_work + P.ell_cls_off[c];
        const int nw = P.ell_cls_n[c], bw = P.ell_cls_w[c], grid = P.ell_cls_grid[c];
        const size_t lds = (size_t)(kBlock / P.group) * bw * sizeof(double);
        FK_DISPATCH_D(P.d, FK_DISPATCH_G(P.group,
            if (f32) k_assemble_ell<float, D, G><<<grid, kBlock, lds, s>>>(P, n, work, nw, bw, org, (float *)vals, (float *)exit_mass);
            else k_assemble_ell<double, D, G><<<grid, kBlock, lds, s>>>(P, n, work, nw, bw, org, (double *)vals, (double *)exit_mass)));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_ell_apply(const PlanDev &P, bool f32, const int *org, const void *vals,
                            const void *exit_mass, const void *packed, void *u_out, hipStream_t s)
{
    FK_DISPATCH_D(P.d,
        if (f32) k_ell_apply<float, D><<<P.row_grid, kBlock, 0, s>>>(P, org, (const float *)vals, (const float *)exit_mass, (const float *)packed, (float *)u_out);
        else k_ell_apply<double, D><<<P.row_grid, kBlock, 0, s>>>(P, org, (const double *)vals, (const double *)exit_mass, (const double *)packed, (double *)u_out));
    return hipGetLastError();
}

hipError_t launch_ell_apply_mc(const PlanDev &P, bool f32, const int *org, const void *vals,
                               const void *exit_mass, const void *packed, long long plane,
                               void *u_out, long long fstride, int nc, hipStream_t s)
{
    if (nc < 1 || nc > 4) return hipErrorInvalidValue;
    FK_DISPATCH_D(P.d,
        if (f32) k_ell_apply_mc<float, D, 4><<<P.row_grid, kBlock, 0, s>>>(P, org, (const float *)vals, (const float *)exit_mass, (const float *)packed, plane, (float *)u_out, fstride, nc);
        else k_ell_apply_mc<double, D, 4><<<P.row_grid, kBlock, 0, s>>>(P, org, (const double *)vals, (const double *)exit_mass, (const double *)packed, plane, (double *)u_out, fstride, nc));
    return hipGetLastError();
}

hipError_t launch_export_ell(const PlanDev &P, bool f32, const int *org_in, const void *vals_in,
                             int *cols_out, void *vals_out, hipStream_t s)
{
    const int g = flat_grid(P.n_active * (long long)P.ell_width);
    FK_DISPATCH_D(P.d,
        if (f32) k_export_ell<float, D><<<g, kBlock, 0, s>>>(P, org_in, (const float *)vals_in, cols_out, (float *)vals_out);
        else k_export_ell<double, D><<<g, kBlock, 0, s>>>(P, org_in, (const double *)vals_in, cols_out, (double *)vals_out));
    return hipGetLastError();
}

hipError_t launch_export_cells(const PlanDev &P, int inst, int n, int *cells,
                               unsigned char *exit_flags, hipStream_t s)
{
    FK_DISPATCH_D(P.d,
        k_export_cells<D><<<4096, kBlock, 0, s>>>(P, inst, n, cells, exit_flags));
    return hipGetLastError();
}

hipError_t launch_clear_flags(const PlanDev &P, hipStream_t s)
{
    k_clear_flags<<<1, 1, 0, s>>>(P.flags);
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const long long n = (long long)(bytes / 4);
    k_zero<<<flat_grid(n), kBlock, 0, s>>>((unsigned int *)p, n);
    return hipGetLastError();
}

hipError_t launch_adjoint_step(const PlanDev &P0, bool f32, int n, const void *packed,
                               const void *lam, void *mu, double *grad, hipStream_t s, int part)
{
    if (P0.step_kind != 1) {
        // part 1: the per-point list only, part 2: the box lists only
        PlanDev P = P0;
        if (part == 1)
            for (int c = 0; c < kBoxClasses; ++c) P.adj.n_box_work[c] = 0;
        if (part == 2) P.adj.n_fw_work = P.adj.n_in_work = 0;
        bool ok = false;
        switch (P.d) {
        case 1: ok = f32 ? adjoint_node_f32_d1(P, n, packed, lam, mu, grad, s) : adjoint_node_f64_d1(P, n, packed, lam, mu, grad, s); break;
        case 2: ok = f32 ? adjoint_node_f32_d2(P, n, packed, lam, mu, grad, s) : adjoint_node_f64_d2(P, n, packed, lam, mu, grad, s); break;
        case 3: ok = f32 ? adjoint_node_f32_d3(P, n, packed, lam, mu, grad, s) : adjoint_node_f64_d3(P, n, packed, lam, mu, grad, s); break;
        default: return hipErrorInvalidValue;
        }
        if (ok) {
            // the staged tiles into mu, once both lists have run
            if (part != 1 && P.adj.stage) {
                FK_DISPATCH_D(P.d,
                    if (f32) k_gather_tiles<float, D><<<flat_grid(P.adj.n_cov), kBlock, 0, s>>>(P.adj.n_cov, P.adj.cov_node, P.adj.cov_ptr, P.adj.cov_base, (const float *)P.adj.stage, (float *)mu);
                    else k_gather_tiles<double, D><<<flat_grid(P.adj.n_cov), kBlock, 0, s>>>(P.adj.n_cov, P.adj.cov_node, P.adj.cov_ptr, P.adj.cov_base, (const double *)P.adj.stage, (double *)mu));
            }
            return hipGetLastError();
        }
    }
    if (part == 2) return hipSuccess;   // the lane-group form has no separate box part
    const PlanDev &P = P0;
    FK_DISPATCH_D(P.d, FK_DISPATCH_G(P.group,
        if (f32) k_adjoint_step<float, D, G><<<P.act_grid, kBlock, 0, s>>>(P, n, (const float *)packed, (const float *)lam, (float *)mu, grad);
        else k_adjoint_step<double, D, G><<<P.act_grid, kBlock, 0, s>>>(P, n, (const double *)packed, (const double *)lam, (double *)mu, grad)));
    return hipGetLastError();
}

hipError_t launch_adjoint_slopes_T(const PlanDev &P, bool f32, const void *u, void *mu,
                                   void *lam_next, hipStream_t s)
{
    // every node an adjoint step can touch lies in the slope pass' node runs
    // (the active region widened by the reach and the slope stencil)
    const WorkItem *runs = P.slope_work;
    const int r0 = P.n_table_work, nr = P.n_slope_work - P.n_table_work;
    if (nr <= 0) return hipSuccess;
    const int g = P.slope_grid;
    FK_DISPATCH_D(P.d,
        if (f32) {
            k_mu_value<float, D><<<g, kBlock, 0, s>>>(P, (float *)mu, (float *)lam_next, runs, r0, nr);
            k_adjoint_slopes_T<float, D><<<g, kBlock, 0, s>>>(P, (const float *)u, (float *)mu, (float *)lam_next, runs, r0, nr);
            k_fold_images<float, D><<<g, kBlock, 0, s>>>(P, (float *)lam_next, runs, r0, nr);
        } else {
            k_mu_value<double, D><<<g, kBlock, 0, s>>>(P, (double *)mu, (double *)lam_next, runs, r0, nr);
            k_adjoint_slopes_T<double, D><<<g, kBlock, 0, s>>>(P, (const double *)u, (double *)mu, (double *)lam_next, runs, r0, nr);
            k_fold_images<double, D><<<g, kBlock, 0, s>>>(P, (double *)lam_next, runs, r0, nr);
        });
    return hipGetLastError();
}

// LDS atomic throughput probe: every lane adds into its own LDS word (no
// bank conflicts, no contention), iters times; one value per workgroup is
// written out so that nothing is dead.
template <typename T>
__global__ void __launch_bounds__(256) k_lds_atomic_probe(int iters, double *out)
{
    __shared__ T buf[256];
    buf[threadIdx.x] = T(0);
    __syncthreads();
    const T v = T(1) + T(threadIdx.x) * T(1e-3);
#pragma unroll 16
    for (int i = 0; i < iters; ++i) atomicAdd(&buf[threadIdx.x], v);
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < 256; ++k) s += (double)buf[k];
        out[blockIdx.x] = s;
    }
}

hipError_t launch_lds_atomic_probe(bool f32, int blocks, int iters, double *out, hipStream_t s)
{
    if (f32) k_lds_atomic_probe<float><<<blocks, 256, 0, s>>>(iters, out);
    else k_lds_atomic_probe<double><<<blocks, 256, 0, s>>>(iters, out);
    return hipGetLastError();
}

hipError_t launch_pack_fields(const PlanDev &P, bool f32, const void *x, void *packed,
                              hipStream_t s)
{
    FK_DISPATCH_D(P.d,
        if (f32) k_pack_fields<float, D><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.n_nodes, (const float *)x, (float *)packed);
        else k_pack_fields<double, D><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.n_nodes, (const double *)x, (double *)packed));
    return hipGetLastError();
}

hipError_t launch_unpack_fields(const PlanDev &P, bool f32, const void *packed, void *x,
                                hipStream_t s)
{
    FK_DISPATCH_D(P.d,
        if (f32) k_unpack_fields<float, D><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.n_nodes, (const float *)packed, (float *)x);
        else k_unpack_fields<double, D><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.n_nodes, (const double *)packed, (double *)x));
    return hipGetLastError();
}

hipError_t launch_masked_diff(const PlanDev &P, bool f32, const void *a, const void *b, void *out,
                              hipStream_t s)
{
    if (f32)
        k_masked_diff<float><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.chi, P.n_nodes, (const float *)a, (const float *)b, (float *)out);
    else
        k_masked_diff<double><<<flat_grid(P.n_nodes), kBlock, 0, s>>>(P.chi, P.n_nodes, (const double *)a, (const double *)b, (double *)out);
    return hipGetLastError();
}

hipError_t launch_convert_out(const PlanDev &P, const double *u, float *out, hipStream_t s)
{
    if (P.n_node_work == 0) return hipSuccess;
    k_convert<true><<<P.node_grid, kBlock, 0, s>>>(P, P.node_work, P.n_node_work,
                                                  const_cast<double *>(u), out);
    return hipGetLastError();
}

hipError_t launch_convert_in(const PlanDev &P, const float *in, double *u, hipStream_t s)
{
    if (P.n_node_work == 0) return hipSuccess;
    k_convert<false><<<P.node_grid, kBlock, 0, s>>>(P, P.node_work, P.n_node_work, u,
                                                   const_cast<float *>(in));
    return hipGetLastError();
}

hipError_t launch_inst_maxdiff(const PlanDev &P, const double *a, const float *b, double *out,
                               hipStream_t s)
{
    if (P.n_node_work == 0) return hipSuccess;
    k_inst_maxdiff<<<P.node_grid, kBlock, 0, s>>>(P, P.node_work, P.n_node_work, a, b,
                                                 (unsigned long long *)out);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(const PlanDev &P, bool f32, const void *lam0, void *lam,
                               hipStream_t s, bool lam0_parent_f32)
{
    hipError_t e = lam0_parent_f32
        ? launch_convert_in(P, (const float *)lam0, (double *)lam, s)
        : hipMemcpyAsync(lam, lam0, (size_t)P.n_nodes * (f32 ? 4 : 8), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    FK_DISPATCH_D(P.d,
        if (f32) k_fold_images<float, D><<<P.node_grid, kBlock, 0, s>>>(P, (float *)lam, P.node_work, 0, P.n_node_work);
        else k_fold_images<double, D><<<P.node_grid, kBlock, 0, s>>>(P, (double *)lam, P.node_work, 0, P.n_node_work));
    return hipGetLastError();
}

}  // namespace fk
