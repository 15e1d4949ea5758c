// Shared declarations of the ensemble backward-Euler step (ensemble_step.hip)
// and its host driver (capi.cpp).
#pragma once
#include <vector>

#include "cfv_kernels.hpp"
#include "cfv_march.hpp"

namespace cfv {

// per instance: device pointers of the step's vectors
struct StepVec {
  const double* U;     // state
  double* Unew;        // output; holds -R during the solve
  double* V;           // (m + 1) Krylov vectors of 9 nc
  double* w;           // work vector, 9 nc
  double* z;           // preconditioned Krylov vector D^-1 V_j (Jacobi), 9 nc
  const double* diag;  // V/dt, nc
  double* sm;          // small per-instance scalars (StepLayout)
  int64_t nc;
  unsigned* flag;      // the instance's status word: bit 1 set when the step's residual norm is not finite
};

// offsets into an instance's scalars for GMRES(m)
struct StepLayout {
  int H, cs, sn, g, y, hcol, beta, kdone, stop, size;
  __host__ __device__ explicit StepLayout(int m) {
    H = 0;                    // (m + 1) x m, row-major
    cs = H + (m + 1) * m;
    sn = cs + m;
    g = sn + m;               // m + 1
    y = g + m + 1;            // m
    hcol = y + m;             // m + 2: the current column of H
    beta = hcol + m + 2;
    kdone = beta + 1;
    stop = kdone + 1;
    size = stop + 1;
  }
};

struct StepLaunch {
  int n, m, blocks;                  // instances, Krylov size, vector blocks per instance
  int precond = 0;                   // 1: GMRES right-preconditioned by the diagonal (Jacobi)
  double cfl;
  const StepVec* sv;                 // device, n
  double* part;                      // device, n x blocks
  double* hist;                      // device, n x m, nullable
  EnsembleLaunch res;                // residual descriptors (output in Unew)
  std::vector<EnsembleLaunch> jvp;   // m JVP descriptor tables (v = V_j, or z with precond; Jv = w)
  std::vector<DevGrid> dev;          // host copies for the per-instance V/dt launches
  std::vector<const double*> Uh;
  std::vector<double*> diagh, Wh;
};

hipError_t launch_ensemble_step(const StepLaunch& L, hipStream_t s, KernelTimer* t);

}  // namespace cfv
