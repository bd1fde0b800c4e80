// Host-side launchers of the BLAS-1 kernels, shared with the solver.
#pragma once

#include "lqcd_internal.h"

namespace lqcd {

int64_t reduce_blocks(const Geom &g, int nhalf);
// partial[2*b], partial[2*b+1] = per-block Re/Im of <a, b> (b != NULL) or |a|^2
void launch_reduce(const Geom &g, int nhalf, const char *a, const char *b, int prec,
                   double *partial, hipStream_t st);
// out[0..nv) = fixed-order sum of n records of nv doubles
void launch_finalize(const double *partial, int64_t n, int nv, double *out, hipStream_t st);
void launch_convert(const Geom &g, int nhalf, char *dst, int pd, const char *src, int ps,
                    hipStream_t st);

}  // namespace lqcd
