// Host-side declarations of the level-1 launchers and the CG scalar block.
#pragma once

#include "wd_internal.h"

namespace wd {

// Largest grid.x of a level-1 launch; reduction partial buffers are sized by it.
constexpr unsigned BLAS_MAX_BLOCKS = 2048;

// Scalars of one CG system; they live in device memory for the whole solve.
struct CgScalars {
  double rr[2];   // |M^dag s|^2, ping-pong between consecutive iterations
  double qq;      // |M p|^2
  double ss;      // |s|^2, s = Schur residual
  double stop2;   // converged when ss <= stop2
  double rnorm2;  // |r|^2 of the FP64 outer residual (defect correction)
  double bb;      // |b|^2
  int done;       // 0 running, 1 converged, 2 breakdown, 3 iteration cap
  int iters;
  int max_iters;
  int pad;
};

// A vector operand: nhalf half fields starting at p; system y at p + y*sys_stride.
struct VecRef {
  const void *p;
  int nhalf;
  size_t sys_stride;
};

inline VecRef vref(const void *p, int nhalf, size_t sys_stride = 0) { return VecRef{p, nhalf, sys_stride}; }

wd_status blas_norm2(const Geom &g, wd_prec prec, const VecRef &x, int nsys, RedBuf red, double *result,
                     hipStream_t st);
wd_status blas_cdot(const Geom &g, wd_prec prec, const VecRef &x, const VecRef &y, int nsys, RedBuf red,
                    double *result, hipStream_t st);
wd_status blas_caxpy(const Geom &g, wd_prec prec, double cre, double cim, const VecRef &x, const VecRef &y,
                     int nsys, hipStream_t st);
// out(po) = scale * x(pi); with sc != NULL the scale is scale / sqrt(sc[sys].rnorm2)
wd_status blas_convert(const Geom &g, wd_prec pi, const VecRef &x, wd_prec po, const VecRef &out, double scale,
                       CgScalars *sc, int nsys, hipStream_t st);
// x64 += scale * sqrt(sc[sys].rnorm2) * e(pe)
wd_status blas_accum(const Geom &g, wd_prec pe, const VecRef &e, const VecRef &x64, double scale, CgScalars *sc,
                     int nsys, hipStream_t st);
wd_status blas_cg_update(const Geom &g, wd_prec px, const VecRef &x, wd_prec pv, const VecRef &p, const VecRef &s,
                         const VecRef &q, CgScalars *sc, int j, int nsys, RedBuf red, hipStream_t st);
wd_status blas_cg_pupdate(const Geom &g, wd_prec pv, const VecRef &r, const VecRef &p, CgScalars *sc, int j,
                          int nsys, hipStream_t st);

}  // namespace wd
