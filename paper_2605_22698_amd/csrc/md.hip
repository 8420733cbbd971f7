// Velocity-Verlet integration in FP64 on the device (Section 1 of the paper:
// batched MD; Appendix H times MD steps). Positions and velocities stay FP64;
// forces arrive in FP32 from the interaction.
//   kick:  v += (dt/2) kappa F / m
//   drift: x += dt v, and flag any atom that moved more than skin/2 since the
//          neighbour lists were built (they must then be rebuilt): the flag
//          takes the maximum of the step stamps that overran, so the host
//          tells a new overrun from an old one without clearing it. The drift
//          also records max over atoms of |x - x_ref| + dt_next |v|, a
//          forecast of the displacement after the next step's drift (the
//          velocity changes little in one step), which lets the host rebuild
//          before an overrun instead of redoing the step after it.
// Langevin dynamics (Section 5.5: the NVT integrator, batched systems with
// independent seeds) adds the Ornstein-Uhlenbeck velocity update of the BAOAB
// splitting,
//   ou:    v <- c1 v + c2 sqrt(kB T kappa / m) z,  c1 = exp(-gamma dt), c2 = sqrt(1 - c1^2)
// with z three standard normals per atom from the Philox4x64-10 counter-based
// generator (Salmon et al., SC'11), key (seed of the atom's structure, 0) and
// counter (step, index of the atom within its structure, 0, 0), turned into
// normals by Box-Muller on the uniforms ((x >> 11) + 1/2) 2^-53. A structure's
// noise is thus independent of what else is packed with it.
#include <algorithm>

#include "common.h"
#include "runtime.h"

namespace e3mi {
namespace {

// Largest forecast of the wave into *probe (non-negative doubles order like
// their bit patterns); one atomic per wave.
__device__ __forceinline__ void record_forecast(double f, unsigned long long* probe) {
  unsigned long long b = __double_as_longlong(f);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(b, off, 64);
    b = o > b ? o : b;
  }
  if ((threadIdx.x & 63) == 0 && b) atomicMax(probe, b);
}

__global__ void k_kick(double* __restrict__ v, const float* __restrict__ F, const int* __restrict__ species,
                       const double* __restrict__ inv_mass, double half_dt_kappa, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double c = half_dt_kappa * inv_mass[species[i]];
  v[3 * i] += c * (double)F[3 * i];
  v[3 * i + 1] += c * (double)F[3 * i + 1];
  v[3 * i + 2] += c * (double)F[3 * i + 2];
}

// Half kick followed by the drift with the kicked velocity (one pass over the
// atoms; the arithmetic of k_kick then k_drift)
__global__ void k_kick_drift(double* __restrict__ v, const float* __restrict__ F, const int* __restrict__ species,
                             const double* __restrict__ inv_mass, double half_dt_kappa, double* __restrict__ x,
                             const double* __restrict__ x_ref, double dt, double limit2, int N,
                             unsigned long long* __restrict__ flag, unsigned long long stamp,
                             unsigned long long* __restrict__ probe, double dt_next) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double forecast = 0.0;
  if (i < N) {
    const double c = half_dt_kappa * inv_mass[species[i]];
    double d2 = 0.0, v2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double vk = v[3 * i + k] + c * (double)F[3 * i + k];
      v[3 * i + k] = vk;
      const double y = x[3 * i + k] + dt * vk;
      x[3 * i + k] = y;
      const double d = y - x_ref[3 * i + k];
      d2 += d * d;
      v2 += vk * vk;
    }
    if (d2 > limit2) atomicMax(flag, stamp);
    forecast = sqrt(d2) + dt_next * sqrt(v2);
  }
  if (probe) record_forecast(forecast, probe);
}

// Half kick; threads below n_copy also copy the structures' energies out.
// v_prev (may be NULL) receives the velocities before the kick, so that the
// step's force evaluation and kick can be redone; probe_clear (may be NULL) is
// zeroed for the next step's forecast.
__global__ void k_kick_copy(double* __restrict__ v, const float* __restrict__ F, const int* __restrict__ species,
                            const double* __restrict__ inv_mass, double half_dt_kappa, int N,
                            const double* __restrict__ e_src, double* __restrict__ e_dst, int n_copy,
                            double* __restrict__ v_prev, unsigned long long* __restrict__ probe_clear) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && probe_clear) *probe_clear = 0;
  if (i < n_copy) e_dst[i] = e_src[i];
  if (i >= N) return;
  const double c = half_dt_kappa * inv_mass[species[i]];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double vk = v[3 * i + k];
    if (v_prev) v_prev[3 * i + k] = vk;
    v[3 * i + k] = vk + c * (double)F[3 * i + k];
  }
}

__global__ void k_drift(double* __restrict__ x, const double* __restrict__ v, const double* __restrict__ x_ref,
                        double dt, double limit2, int N, unsigned long long* __restrict__ flag,
                        unsigned long long stamp, unsigned long long* __restrict__ probe, double dt_next) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double forecast = 0.0;
  if (i < N) {
    double d2 = 0.0, v2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double vk = v[3 * i + k];
      const double y = x[3 * i + k] + dt * vk;
      x[3 * i + k] = y;
      const double d = y - x_ref[3 * i + k];
      d2 += d * d;
      v2 += vk * vk;
    }
    if (d2 > limit2) atomicMax(flag, stamp);
    forecast = sqrt(d2) + dt_next * sqrt(v2);
  }
  if (probe) record_forecast(forecast, probe);
}

__global__ void k_nonfinite(const double* __restrict__ x, int n, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!isfinite(x[i])) atomicOr(flag, 4);
}

// Species outside [0, n_species) would index past the per-species tables
__global__ void k_species_range(const int* __restrict__ species, int n, int n_species, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int z = species[i];
  if (z < 0 || z >= n_species) atomicOr(flag, 8);
}

// Philox4x64 block function, 10 rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
    const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += W0;
    k1 += W1;
  }
}

__global__ void k_ou(double* __restrict__ v, const int* __restrict__ species, const double* __restrict__ inv_mass,
                     const int* __restrict__ owner, const int64_t* __restrict__ offsets,
                     const uint64_t* __restrict__ seeds, const int64_t* __restrict__ step0, int64_t step, double c1,
                     double c2, double kT_kappa, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int s = owner[i];
  uint64_t c[4] = {(uint64_t)(step0[s] + step), (uint64_t)(i - offsets[s]), 0ull, 0ull};
  philox4x64_10(c, seeds[s], 0ull);
  constexpr double two53 = 1.0 / 9007199254740992.0;
  double u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = ((double)(c[k] >> 11) + 0.5) * two53;
  constexpr double two_pi = 6.283185307179586476925286766559;
  const double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
  const double z0 = r0 * cos(two_pi * u[1]), z1 = r0 * sin(two_pi * u[1]), z2 = r1 * cos(two_pi * u[3]);
  const double sig = c2 * sqrt(kT_kappa * inv_mass[species[i]]);
  v[3 * i] = c1 * v[3 * i] + sig * z0;
  v[3 * i + 1] = c1 * v[3 * i + 1] + sig * z1;
  v[3 * i + 2] = c1 * v[3 * i + 2] + sig * z2;
}

// Monte Carlo barostat: scale a structure's positions by its factor, and
// put back the rows of the structures whose volume move was rejected.
__global__ void k_scale_positions(double* __restrict__ x, const int* __restrict__ owner, const double* __restrict__ lam,
                                  int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double f = lam[owner[i]];
  x[3 * i] *= f;
  x[3 * i + 1] *= f;
  x[3 * i + 2] *= f;
}

__global__ void k_restore_rows(double* __restrict__ x, const double* __restrict__ x_save, const int* __restrict__ owner,
                               const int* __restrict__ keep, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N || keep[owner[i]]) return;
  x[3 * i] = x_save[3 * i];
  x[3 * i + 1] = x_save[3 * i + 1];
  x[3 * i + 2] = x_save[3 * i + 2];
}

__global__ void k_zero(unsigned* __restrict__ p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0u;
}

inline int blocks(long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_kick(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa, int N,
                 hipStream_t st) {
  if (N == 0) return;
  k_kick<<<blocks(N, 256), 256, 0, st>>>(v, F, species, inv_mass, half_dt_kappa, N);
}
void launch_kick_drift(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa,
                       double* x, const double* x_ref, double dt, double limit2, int N, unsigned long long* flag,
                       unsigned long long stamp, unsigned long long* probe, double dt_next, hipStream_t st) {
  if (N == 0) return;
  k_kick_drift<<<blocks(N, 256), 256, 0, st>>>(v, F, species, inv_mass, half_dt_kappa, x, x_ref, dt, limit2, N, flag,
                                               stamp, probe, dt_next);
}
void launch_kick_copy(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa,
                      int N, const double* e_src, double* e_dst, int n_copy, double* v_prev,
                      unsigned long long* probe_clear, hipStream_t st) {
  const int n = std::max(std::max(N, n_copy), probe_clear ? 1 : 0);
  if (n == 0) return;
  k_kick_copy<<<blocks(n, 256), 256, 0, st>>>(v, F, species, inv_mass, half_dt_kappa, N, e_src, e_dst, n_copy,
                                              v_prev, probe_clear);
}
void launch_drift(double* x, const double* v, const double* x_ref, double dt, double limit2, int N,
                  unsigned long long* flag, unsigned long long stamp, unsigned long long* probe, double dt_next,
                  hipStream_t st) {
  if (N == 0) return;
  k_drift<<<blocks(N, 256), 256, 0, st>>>(x, v, x_ref, dt, limit2, N, flag, stamp, probe, dt_next);
}
void launch_ou(double* v, const int* species, const double* inv_mass, const int* owner, const int64_t* offsets,
               const uint64_t* seeds, const int64_t* step0, int64_t step, double c1, double c2, double kT_kappa, int N,
               hipStream_t st) {
  if (N == 0) return;
  k_ou<<<blocks(N, 256), 256, 0, st>>>(v, species, inv_mass, owner, offsets, seeds, step0, step, c1, c2, kT_kappa, N);
}
void launch_scale_positions(double* x, const int* owner, const double* lam, int N, hipStream_t st) {
  if (N == 0) return;
  k_scale_positions<<<blocks(N, 256), 256, 0, st>>>(x, owner, lam, N);
}
void launch_restore_rows(double* x, const double* x_save, const int* owner, const int* keep, int N, hipStream_t st) {
  if (N == 0) return;
  k_restore_rows<<<blocks(N, 256), 256, 0, st>>>(x, x_save, owner, keep, N);
}
void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const long n = (long)(bytes / 4);
  if (n == 0) return;
  k_zero<<<std::min(blocks(n, 256), 4096), 256, 0, st>>>(static_cast<unsigned*>(p), n);
}
void launch_nonfinite(const double* x, int n, int* flag, hipStream_t st) {
  if (n == 0) return;
  k_nonfinite<<<blocks(n, 256), 256, 0, st>>>(x, n, flag);
}
void launch_species_range(const int* species, int n, int n_species, int* flag, hipStream_t st) {
  if (n == 0) return;
  k_species_range<<<blocks(n, 256), 256, 0, st>>>(species, n, n_species, flag);
}

}  // namespace e3mi
