// hh_setup.h -- host-side setup of one grid: node maps, Shortley-Weller
// coefficients, coarse phi, explicit inverse of the coarsest preconditioner.
#pragma once
#include <string>
#include <vector>

#include "hh_common.h"
#include "../../include/hh.h"

struct HostLevel {
    int n[3] = {1, 1, 1};
    int64_t N = 1;
    std::vector<double2> aM[3], cM[3], dM[3];
    std::vector<double> phi;
    std::vector<double2> gal;     // Galerkin levels >= 1: 25 x N stencil, entry s = (dx+2) + 5(dy+2)
                                  // of point p at s*N + p (the matrix entry M[p, p + dx + nx*dy])
    std::vector<double2> ilu;     // ILU(0) smoothing levels: 25 x N factors in the same layout
                                  // (L below the diagonal, unit diagonal not stored; U on and above)
};

struct HostSetup {
    int dim = 2, nlev = 1;
    int centering = HH_CELL;                    // HH_VERTEX: one level, no hierarchy
    int nu1 = 1;                                // pre-smoothing steps: 1 (V(1,1)) or 0 (V(0,1))
    int coarse_op = HH_COARSE_REDISCRETISED;    // HH_COARSE_GALERKIN: levels >= 1 carry gal
    int smoother = HH_SMOOTH_JACOBI;            // HH_SMOOTH_ILU0: levels 0 .. nlev-2 carry ilu
    double omega = 0.8;
    std::vector<double2> aH[3], cH[3], dH[3];   // finest level, ECS operator
    HostLevel lev[HH_MAXLEV];
    int Nc = 0;
    std::vector<double2> Minv;                  // Nc x Nc row major
};

// Validates a description without building anything: levels (the automatic
// rule applied) and coarsest unknowns.  phi is not read.
hh_status desc_check(const hh_grid_desc *d, int &levels, int &coarse, std::string &err);

// Validates the description and fills hs.  Returns HH_OK or HH_ERR_ARG with
// a message in err.
hh_status host_setup(const hh_grid_desc *d, HostSetup &hs, std::string &err);

// Number of levels the automatic rule picks for sides n[0..dim).
int auto_levels(int dim, const int *n);

// Host evaluation of y = M x on one level (used to build the coarse matrix and
// the Galerkin operators): the rediscretised stencil, or the level's Galerkin
// stencil when it has one.
void host_apply_M(const HostSetup &hs, int lev, const double2 *x, double2 *y);
