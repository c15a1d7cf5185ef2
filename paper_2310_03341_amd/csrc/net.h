// Start-field network (learned SCF start): layout and entry points.
#pragma once
#include "common.h"

namespace bdg {

struct NetLayout {
    int64_t w_off[4], b_off[4], nparams;
    int cin[4], cout[4];
    size_t wk[4], wt[4], act[4], y, g32, gbf, gx32, part, total;
};

NetLayout net_layout(const bdg_net_shape *sh, bool forward_only = false);
int net_forward(const bdg_net_shape *sh, const float *params, const double *Vext, const double *theta,
                double mu, float *y_out, void *work, hipStream_t s);
int net_forward_noalloc(const bdg_net_shape *sh, const float *params, const double *Vext, const double *theta,
                        double mu, float *y_out, hipStream_t s);
size_t net_scratch_capacity();
int net_backward(const bdg_net_shape *sh, const float *params, const double *Vext, const double *theta,
                 double mu, const float *target, float *grads, float *loss, void *work, hipStream_t s);
int net_start_fields(const bdg_net_shape *sh, const float *y, int sample, const double *Vext, double *U, double *D,
                     hipStream_t s);
int net_adam(int64_t np, float *params, const float *grads, float *m, float *v, int t, float lr,
             hipStream_t s);

}  // namespace bdg
