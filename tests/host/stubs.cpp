// Stand-ins for the kernel launchers (defined in the HIP sources) so that the
// planner links into a host-only program.  The host checks never reach them;
// if one is called it reports a launch failure.
#include <hip/hip_runtime.h>

#include "slos_internal.h"
#include "slos_ext.h"

static int no_launch() { return 1; }
int slos_launch_cdf(const void *, int, int64_t, double *, void *) { return no_launch(); }
int slos_launch_seed(const void *, uint64_t, uint32_t, const double *, const void *, void *, int, void *, int, uint64_t,
                     uint64_t) { return no_launch(); }
int slos_launch_batch(const BatchParams &, int, int, int, int, void *) { return no_launch(); }
int slos_launch_colsum_gradu(const void *, const ColsumLayers &, const int32_t *, int, int, void *, int, void *, int,
                             uint64_t, uint64_t)
{
    return no_launch();
}
int slos_launch_sq_loss(const void *, uint64_t, const int64_t *, int64_t, const double *, void *, double *, int, int,
                        void *)
{
    return no_launch();
}
int slos_launch_sq_loss_seed(const void *, uint64_t, const int64_t *, const double *, int64_t, const double *, void *,
                             uint64_t, double *, int, int, void *)
{
    return no_launch();
}
int slos_launch_layer(const LayerParams &, const LayerLaunch &, void *) { return no_launch(); }
int slos_launch_reduce(const double *, int64_t, double *, double *, void *, int, int64_t) { return no_launch(); }
int slos_launch_sample(const void *, int, int64_t, const double *, const double *, int64_t, int64_t *, void *)
{
    return no_launch();
}
int slos_launch_select(const SelectParams &, int, void *) { return no_launch(); }
int slos_launch_vacuum(void *, int, int, double *, void *) { return no_launch(); }
int slos_launch_src_fill(const SrcFillParams &, int, void *) { return no_launch(); }
int slos_launch_src_pass(const SrcPassParams &, int, void *) { return no_launch(); }
int slos_launch_zero_u32(uint32_t *, int, void *) { return no_launch(); }
int slos_launch_bwd_layer(const BwdParams &, int, int, void *, int) { return no_launch(); }
int slos_launch_marginals(const void *, int, const double *, const int64_t *, int, double *, void *)
{
    return no_launch();
}
int slos_launch_src_group(const SrcGroupParams &, int, void *) { return no_launch(); }
int slos_launch_src_stats(const SrcStatsParams &, void *) { return no_launch(); }
int slos_launch_postselect(const PostselectParams &, int, void *) { return no_launch(); }
int slos_launch_mesh_forward(int, int, const double *, void *, int, void *) { return no_launch(); }
int slos_launch_mesh_backward(int, int, const double *, const void *, double *, int, void *) { return no_launch(); }
int slos_prepare_batch_kernels() { return no_launch(); }
int slos_launch_postselect_table(const PostselectParams &, int, const int64_t *, int64_t, const double *, double *,
                                 void *)
{
    return no_launch();
}
int slos_static_scratch(void **, int *) { return no_launch(); }
