// Host-side launchers of the library's kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace gabp {

// dtype: 0 = FP32 message planes, 1 = FP64.
hipError_t launch_iter(int dtype, const Lattice &L, const void *min, void *mout,
                       const void *adiag, const void *bw, double eta, uint32_t *flag,
                       uint32_t t, hipStream_t s);
hipError_t launch_post(int dtype, const Lattice &L, const void *m, const double *adiag64,
                       const double *b64, double *mu_plane, double *mean, double *var,
                       hipStream_t s);
hipError_t launch_resid(const Lattice &L, const double *mu, const double *adiag64,
                        const double *b64, double *partials, int npart, double *out,
                        hipStream_t s);
hipError_t launch_abs_change(int dtype, const void *a, const void *b, int64_t n,
                             double *partials, int npart, double *out, hipStream_t s);
hipError_t launch_setup(int dtype, const Lattice &L, int64_t nobs, const int64_t *cell,
                        const double *y, const double *var, double sigma2, double *adiag64,
                        double *b64, const double *prior_mean, void *adiag_w, void *b_w,
                        uint32_t *err_flag, hipStream_t s);
hipError_t launch_msgs_get(int dtype, const Lattice &L, const void *m, void *prec, void *info,
                           hipStream_t s);
hipError_t launch_msgs_set(int dtype, const Lattice &L, void *m, const void *prec,
                           const void *info, hipStream_t s);

}  // namespace gabp
