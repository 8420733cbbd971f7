// Long-range electrostatics of open structures (Section 5.1, the
// charge-correction and long-range-interaction equations):
//   raw charges   q_i = w_q . h_i[0] + b_q[z_i]      (written by the readout)
//   correction    q~_i = q_i - (sum_{j in s} q_j - Q_s) / N_s
//   energy        E_i += 1/2 k_e q~_i phi_i,   phi_i = sum_{j != i in s} q~_j kappa(r_ij)
//   kappa(r) = 1/chi(r) = f(r/r0) / sqrt(r^2 + 1) + (1 - f(r/r0)) / r,
//   f(x) = 1 - 6x^5 + 15x^4 - 10x^3 for x < 1, else 0   (PhysNet's soft core)
// and its adjoint:
//   F_i  += k_e q~_i sum_j q~_j kappa'(r_ij) (r_j - r_i) / r_ij
//   dE/dq_i = k_e (phi_i - mean_{k in s} phi_k)          (through the correction)
//   dE/dh_i[0] += dE/dq_i w_q                            (into the readout's adjoint)
// All pairs of a structure, no cutoff: O(N_s^2) per structure. One 64-lane
// workgroup per tile of 64 receivers of one structure; sender positions and
// charges are staged through LDS 64 at a time, so each sender is read from
// HBM once per tile. Positions are taken relative to the structure's first
// atom in FP64 before rounding to FP32; the potential sum is kept in FP64.
#include "common.h"
#include "runtime.h"

namespace e3mi {
namespace {

constexpr float kCoulombK = 14.399645478425668f;  // e^2 / (4 pi eps0) in eV angstrom

__device__ __forceinline__ double block_sum_256(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// One block of 256 threads per structure: q~ = q - (sum q - Q_s) / N_s.
__global__ void __launch_bounds__(256) k_charge_fix(const float* __restrict__ q_raw, const int64_t* __restrict__ off,
                                                    const double* __restrict__ Q, float* __restrict__ q) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  if (b == a) return;
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) acc += (double)q_raw[i];
  const double tot = block_sum_256(acc, red);
  const double shift = (tot - Q[s]) / (double)(b - a);
  for (int64_t i = a + threadIdx.x; i < b; i += 256) q[i] = (float)((double)q_raw[i] - shift);
}

// Tile t covers receivers tiles[t].y .. +63 of structure tiles[t].x.
__global__ void __launch_bounds__(64) k_coulomb(const int2* __restrict__ tiles, const int64_t* __restrict__ off,
                                                const double* __restrict__ pos, const float* __restrict__ q,
                                                float inv_r0, double* __restrict__ e_atom, float* __restrict__ pot,
                                                float* __restrict__ fc) {
  __shared__ float4 xs[64];
  const int2 tl = tiles[blockIdx.x];
  const int64_t a = off[tl.x], b = off[tl.x + 1];
  const int lane = threadIdx.x;
  const int64_t i = (int64_t)tl.y + lane;
  const bool live = i < b;
  const double ox = pos[3 * a], oy = pos[3 * a + 1], oz = pos[3 * a + 2];
  float xi = 0.f, yi = 0.f, zi = 0.f;
  if (live) {
    xi = (float)(pos[3 * i] - ox);
    yi = (float)(pos[3 * i + 1] - oy);
    zi = (float)(pos[3 * i + 2] - oz);
  }
  double phi = 0.0;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  for (int64_t j0 = a; j0 < b; j0 += 64) {
    const int64_t j = j0 + lane;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j < b)
      v = make_float4((float)(pos[3 * j] - ox), (float)(pos[3 * j + 1] - oy), (float)(pos[3 * j + 2] - oz), q[j]);
    __syncthreads();
    xs[lane] = v;
    __syncthreads();
    const int m = (int)min((int64_t)64, b - j0);
    const int kself = (int)max((int64_t)-1, min((int64_t)64, i - j0));  // the receiver's own slot, if here
    float ps = 0.f;
    for (int k = 0; k < m; ++k) {
      const float4 s = xs[k];
      const float dx = s.x - xi, dy = s.y - yi, dz = s.z - zi;
      const bool self = k == kself;
      const float r2 = self ? 1.0f : dx * dx + dy * dy + dz * dz;
      const float qj = self ? 0.0f : s.w;
      const float rinv = rsqrtf(r2);
      const float r = r2 * rinv;
      const float x = fminf(r * inv_r0, 1.0f);
      const float om = 1.0f - x;
      const float f = 1.0f + x * x * x * (-10.0f + x * (15.0f - 6.0f * x));
      const float df = -30.0f * inv_r0 * x * x * om * om;
      const float sr = rsqrtf(r2 + 1.0f);
      const float kap = rinv + f * (sr - rinv);
      const float dkap = df * (sr - rinv) - f * r * sr * sr * sr - (1.0f - f) * rinv * rinv;
      ps += qj * kap;
      const float gq = qj * dkap * rinv;
      fx += gq * dx;
      fy += gq * dy;
      fz += gq * dz;
    }
    phi += (double)ps;
  }
  if (!live) return;
  const float qi = q[i];
  e_atom[i] += 0.5 * (double)kCoulombK * (double)qi * phi;
  pot[i] = (float)((double)kCoulombK * phi);
  const float c = kCoulombK * qi;
  fc[3 * i] = c * fx;
  fc[3 * i + 1] = c * fy;
  fc[3 * i + 2] = c * fz;
}

// One block of 256 threads per structure: dh_i[k] += (pot_i - mean pot) w_q[k].
__global__ void __launch_bounds__(256) k_coulomb_dq(const int64_t* __restrict__ off, const float* __restrict__ pot,
                                                    const float* __restrict__ wq, int C, float* __restrict__ dh) {
  __shared__ double red[256];
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  if (b == a) return;
  double acc = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) acc += (double)pot[i];
  const float mean = (float)(block_sum_256(acc, red) / (double)(b - a));
  for (int64_t e = a * C + threadIdx.x; e < b * C; e += 256) {
    const int64_t i = e / C;
    const int k = (int)(e - i * C);
    dh[e] += (pot[i] - mean) * wq[k];
  }
}

}  // namespace

void launch_charge_fix(const float* q_raw, const int64_t* off, const double* Q, int S, float* q, hipStream_t st) {
  if (S == 0) return;
  k_charge_fix<<<S, 256, 0, st>>>(q_raw, off, Q, q);
}

void launch_coulomb(const int2* tiles, int n_tiles, const int64_t* off, const double* pos, const float* q, float r0,
                    double* e_atom, float* pot, float* fc, hipStream_t st) {
  if (n_tiles == 0) return;
  k_coulomb<<<n_tiles, 64, 0, st>>>(tiles, off, pos, q, 1.0f / r0, e_atom, pot, fc);
}

void launch_coulomb_dq(const int64_t* off, int S, const float* pot, const float* wq, int C, float* dh,
                       hipStream_t st) {
  if (S == 0) return;
  k_coulomb_dq<<<S, 256, 0, st>>>(off, pot, wq, C, dh);
}

}  // namespace e3mi
