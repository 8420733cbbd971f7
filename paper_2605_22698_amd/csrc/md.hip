// Velocity-Verlet integration in FP64 on the device (Section 1 of the paper:
// batched MD; Appendix H times MD steps). Positions and velocities stay FP64;
// forces arrive in FP32 from the interaction.
//   kick:  v += (dt/2) kappa F / m
//   drift: x += dt v, and flag any atom that moved more than skin/2 since the
//          neighbour lists were built (they must then be rebuilt)
#include "common.h"
#include "runtime.h"

namespace e3mi {
namespace {

__global__ void k_kick(double* __restrict__ v, const float* __restrict__ F, const int* __restrict__ species,
                       const double* __restrict__ inv_mass, double half_dt_kappa, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double c = half_dt_kappa * inv_mass[species[i]];
  v[3 * i] += c * (double)F[3 * i];
  v[3 * i + 1] += c * (double)F[3 * i + 1];
  v[3 * i + 2] += c * (double)F[3 * i + 2];
}

__global__ void k_drift(double* __restrict__ x, const double* __restrict__ v, const double* __restrict__ x_ref,
                        double dt, double limit2, int N, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double d2 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double y = x[3 * i + k] + dt * v[3 * i + k];
    x[3 * i + k] = y;
    const double d = y - x_ref[3 * i + k];
    d2 += d * d;
  }
  if (d2 > limit2) atomicOr(flag, 1);
}

__global__ void k_nonfinite(const double* __restrict__ x, int n, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!isfinite(x[i])) atomicOr(flag, 4);
}

inline int blocks(long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_kick(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa, int N,
                 hipStream_t st) {
  if (N == 0) return;
  k_kick<<<blocks(N, 256), 256, 0, st>>>(v, F, species, inv_mass, half_dt_kappa, N);
}
void launch_drift(double* x, const double* v, const double* x_ref, double dt, double limit2, int N, int* flag,
                  hipStream_t st) {
  if (N == 0) return;
  k_drift<<<blocks(N, 256), 256, 0, st>>>(x, v, x_ref, dt, limit2, N, flag);
}
void launch_nonfinite(const double* x, int n, int* flag, hipStream_t st) {
  if (n == 0) return;
  k_nonfinite<<<blocks(n, 256), 256, 0, st>>>(x, n, flag);
}

}  // namespace e3mi
