// snap_kernels.hpp -- launch interface between the C ABI and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "snap_tables.hpp"

namespace snapmi {

struct Geom {
    double rcut, rfac0, rmin0, wself;
    double box[3];
    int switch_flag;
};

// Device copies of the tables of one context.
struct DevTables {
    double *unscale_u = nullptr, *unscale_y = nullptr;
    Term *terms = nullptr;
    ZItem *items = nullptr;
    YRow *rows = nullptr;
    BItem *bitems = nullptr;
    int *bl_begin = nullptr;
    int nrows = 0;
};

// Per-call device workspace.  Per-atom arrays are element-major:
// X[e * npad + atom], npad = n rounded up to 64.
struct Work {
    double2 *U = nullptr, *Y = nullptr;
    double *dE = nullptr;
    int *pair_atom = nullptr;
    int *flag = nullptr;
    int npad = 0;
};

hipError_t launch_compute_u(int twojmax, int n, int npad, const double *pos, const int *off,
                            const int *nbr, const DevTables &T, const Geom &g, double2 *U,
                            int *pair_atom, int *flag, hipStream_t s);

hipError_t launch_compute_y(int n, int npad, int nhalf, const double2 *U, double2 *Y,
                            const DevTables &T, const double *beta, int per_atom_beta, int nb,
                            const double *gscale, hipStream_t s);

hipError_t launch_bispectrum(int n, int npad, const double2 *U, const DevTables &T, int nb,
                             double *B, const double *beta, int per_atom_beta, double *energy,
                             hipStream_t s);

hipError_t launch_dedr(int twojmax, int dirs, int npairs, int npad, const double *pos,
                       const int *nbr, const int *pair_atom, const double2 *Y, const DevTables &T,
                       const Geom &g, double *dE, hipStream_t s);

hipError_t launch_gather(int n, int npad, int nhalf, const int *off, const int *rev,
                         const double *dE, const double2 *U, const double2 *Y, double *energy,
                         double *force, hipStream_t s);

// dst[e][atom][re/im] = scale[e] * src[e * npad + atom] for atom < n
hipError_t launch_unscale(int n, int npad, int nhalf, const double2 *src, const double *scale,
                          double *dst, hipStream_t s);

}  // namespace snapmi
