// Host-callable launchers of the gfx950 kernels (defined in hmc_kernels.hip).
// P selects the number format (0 FP64, 1 FP32, 2 BF16); R is the row-tile
// height (16, 32 or 64).
#pragma once
#include <hip/hip_runtime.h>
#include "hmc_plan.hpp"

hipError_t hmc_set_lds_limit(int P, int R, size_t lds_bytes);
hipError_t hmc_launch_mlp_grad(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t hmc_launch_trunk_fwd(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t hmc_launch_branch_grad(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t hmc_launch_trunk_bwd(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t hmc_launch_mlp_energy(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t hmc_launch_branch_energy(int P, int R, int nt, const GradArgs& a, int grid, size_t lds, hipStream_t s);
hipError_t hmc_launch_tower_sens(int P, int R, int nt, const GradArgs& a, int tower, const void* seed, int grid,
                                 size_t lds, hipStream_t s);
hipError_t hmc_launch_tower_out(int P, int R, int nt, const GradArgs& a, int tower, void* out, int ld, int grid,
                                size_t lds, hipStream_t s);
hipError_t hmc_launch_sens_reduce(int P, const void* part, int tiles, long long n, long long k0, long long k1,
                                  double* acc, const double* sigma, double inv_nd, double* s2, hipStream_t s);
hipError_t hmc_launch_mlp_predict(int P, int R, int nt, const GradArgs& a, int c, int grid, size_t lds,
                                  hipStream_t s, double* mean, double* m2, double* var, double inv_k, double inv_n);
hipError_t hmc_launch_combine_predict(int P, const void* Bn, const void* Tn, int ld, int p, long long nu, long long nq,
                                     const void* b0, double* mean, double* m2, double* var, double inv_k,
                                     double inv_n, hipStream_t s);
hipError_t hmc_launch_zero(double* p, long long n, hipStream_t s);
hipError_t hmc_launch_scatter_vec(int P, const StateArgs& sa, int c, const void* vec, long long n, hipStream_t s);
hipError_t hmc_launch_update(int P, const StateArgs& s, int mode, int gx, int sub, hipStream_t st);
hipError_t hmc_launch_update_split(int P, const StateArgs& s, int mode, int gx, hipStream_t st);
hipError_t hmc_launch_traj_begin(int P, const StateArgs& s, hipStream_t st);
hipError_t hmc_launch_traj_end(int P, const StateArgs& s, int mode, hipStream_t st);
hipError_t hmc_launch_momentum(int P, const StateArgs& s, hipStream_t st);
hipError_t hmc_launch_restore(int P, const StateArgs& s, hipStream_t st);
hipError_t hmc_launch_scatter_all(int P, const StateArgs& s, hipStream_t st);
