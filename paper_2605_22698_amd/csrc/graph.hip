// Neighbour lists on the GPU (Section 3.2 of the paper: the graph of a chemical
// system is all pairs within a cutoff radius, with periodic images).
//
// Build (every few MD steps):
//   owner/bbox -> cell grid per structure (host plan) -> bin atoms into cells
//   -> per-receiver stencil scan, two passes (count, fill) -> per-row sort of
//   (j, n) keys -> reverse-edge index by binary search.
// Per energy evaluation:
//   prune the skin list to r < r_c (count per row, scan, compact, remap the
//   reverse index), writing the FP32 edge vectors the interaction consumes.
//
// Edge key: (uint64)j << 24 | (nx+128) << 16 | (ny+128) << 8 | (nz+128),
// so sorting keys sorts by (j, nx, ny, nz); the low 24 bits are the packed
// image vector stored per edge.
#include "common.h"
#include "runtime.h"

namespace e3mi {

namespace {

__device__ __forceinline__ int unpack_n(int s, int axis) { return ((s >> (16 - 8 * axis)) & 255) - 128; }

__global__ void k_owner(const int64_t* __restrict__ off, int* __restrict__ owner) {
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x) owner[i] = s;
}

__global__ void k_bbox(const double* __restrict__ pos, const int64_t* __restrict__ off,
                       double* __restrict__ bbox) {
  const int s = blockIdx.x;
  const int64_t a = off[s], b = off[s + 1];
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = a + threadIdx.x; i < b; i += blockDim.x)
    for (int k = 0; k < 3; ++k) {
      const double v = pos[3 * i + k];
      mn[k] = fmin(mn[k], v);
      mx[k] = fmax(mx[k], v);
    }
  __shared__ double red[6][256];
  for (int k = 0; k < 3; ++k) {
    red[k][threadIdx.x] = mn[k];
    red[3 + k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + w]);
        red[3 + k][threadIdx.x] = fmax(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) bbox[6 * s + threadIdx.x] = red[threadIdx.x][0];
}

// Single-workgroup exclusive scan; out has n + 1 entries (out[n] = total).
// Tiles of 4 x 1024 elements, each scanned by the block and carried forward.
__global__ void __launch_bounds__(1024) k_exclusive_scan(const int* __restrict__ in, int* __restrict__ out, int n) {
  __shared__ int wsum[16];
  __shared__ int carry_s;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < n; base += 4096) {
    int v[4];
    int local = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = base + 4 * t + k;
      v[k] = idx < n ? in[idx] : 0;
      local += v[k];
    }
    // inclusive wave scan of `local`
    int x = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (t < 16) {
      int s = wsum[t];
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const int y = __shfl_up(s, off, 16);
        if (t >= off) s += y;
      }
      wsum[t] = s;  // inclusive over waves
    }
    __syncthreads();
    const int carry = carry_s;
    int run = carry + (w ? wsum[w - 1] : 0) + x - local;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int idx = base + 4 * t + k;
      if (idx < n) out[idx] = run;
      run += v[k];
    }
    __syncthreads();
    if (t == 1023) carry_s = run;
    __syncthreads();
  }
  if (t == 0) out[n] = carry_s;
}

__device__ __forceinline__ int floor_div(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// Wrapped coordinate, image offset and cell index along one axis.
__device__ __forceinline__ void wrap_axis(double x, const GridPlan& g, int k, double& w, int& a, int& c) {
  if (g.periodic[k]) {
    const double f = floor(x / g.len[k]);
    a = (int)f;
    w = x - f * g.len[k];
  } else {
    a = 0;
    w = x - g.lo[k];
  }
  c = (int)floor(w * g.inv_cw[k]);
  c = c < 0 ? 0 : (c >= g.nb[k] ? g.nb[k] - 1 : c);
}

__global__ void k_bin(const double* __restrict__ pos, const int* __restrict__ owner,
                      const GridPlan* __restrict__ plan, int N, int* __restrict__ atom_cell,
                      int* __restrict__ wrap, int* __restrict__ cell_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const GridPlan g = plan[owner[i]];
  int c[3];
  for (int k = 0; k < 3; ++k) {
    double w;
    int a;
    wrap_axis(pos[3 * i + k], g, k, w, a, c[k]);
    wrap[3 * i + k] = a;
  }
  const int cell = g.cell_base + (c[0] * g.nb[1] + c[1]) * g.nb[2] + c[2];
  atom_cell[i] = cell;
  atomicAdd(&cell_count[cell], 1);
}

__global__ void k_bin_fill(const int* __restrict__ atom_cell, const int* __restrict__ cell_start, int N,
                           int* __restrict__ cell_fill, int* __restrict__ cell_atoms) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int c = atom_cell[i];
  const int slot = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + slot] = i;
}

// One thread per receiver: scan the cells whose unwrapped index range covers
// [w_i - rc, w_i + rc] on every axis; each unwrapped cell u maps to the cell
// u mod nb and the image floor(u / nb), so no (j, n) pair is visited twice.
// One wave per receiver: the lanes scan the atoms of each stencil cell
// together; hits are compacted with a ballot, so a row's edges are found in
// the same order in the counting and the filling pass.
template <bool FILL>
__global__ void __launch_bounds__(256) k_edges(const double* __restrict__ pos, const int* __restrict__ owner,
                                               const GridPlan* __restrict__ plan, const int* __restrict__ wrap,
                                               const int* __restrict__ cell_start, const int* __restrict__ cell_atoms,
                                               const int* __restrict__ row_ptr, int N, double rc2,
                                               int* __restrict__ count, uint64_t* __restrict__ keys,
                                               int* __restrict__ err) {
  const int i = (int)(((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= N) return;  // the whole wave leaves together
  const GridPlan g = plan[owner[i]];
  const double rc = sqrt(rc2);
  const double xi[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
  const int ai[3] = {wrap[3 * i], wrap[3 * i + 1], wrap[3 * i + 2]};
  int ulo[3], uhi[3];
  for (int k = 0; k < 3; ++k) {
    double w;
    int a, c;
    wrap_axis(xi[k], g, k, w, a, c);
    const double eps = 1e-6;
    ulo[k] = (int)floor((w - rc - eps) * g.inv_cw[k]);
    uhi[k] = (int)floor((w + rc + eps) * g.inv_cw[k]);
    if (!g.periodic[k]) {
      ulo[k] = ulo[k] < 0 ? 0 : ulo[k];
      uhi[k] = uhi[k] > g.nb[k] - 1 ? g.nb[k] - 1 : uhi[k];
    }
  }
  const uint64_t below = (1ull << lane) - 1ull;
  int n_found = 0;
  const int base = FILL ? row_ptr[i] : 0;
  for (int ux = ulo[0]; ux <= uhi[0]; ++ux) {
    const int cx = ux - floor_div(ux, g.nb[0]) * g.nb[0], nwx = g.periodic[0] ? floor_div(ux, g.nb[0]) : 0;
    for (int uy = ulo[1]; uy <= uhi[1]; ++uy) {
      const int cy = uy - floor_div(uy, g.nb[1]) * g.nb[1], nwy = g.periodic[1] ? floor_div(uy, g.nb[1]) : 0;
      for (int uz = ulo[2]; uz <= uhi[2]; ++uz) {
        const int cz = uz - floor_div(uz, g.nb[2]) * g.nb[2], nwz = g.periodic[2] ? floor_div(uz, g.nb[2]) : 0;
        const int cell = g.cell_base + (cx * g.nb[1] + cy) * g.nb[2] + cz;
        const int b0 = cell_start[cell], b1 = cell_start[cell + 1];
        for (int q0 = b0; q0 < b1; q0 += 64) {
          const int q = q0 + lane;
          bool hit = false;
          uint64_t key = 0;
          if (q < b1) {
            const int j = cell_atoms[q];
            // image vector for the raw positions: r_j - r_i + n.L
            const int n0 = nwx + ai[0] - wrap[3 * j];
            const int n1 = nwy + ai[1] - wrap[3 * j + 1];
            const int n2 = nwz + ai[2] - wrap[3 * j + 2];
            const double dx = (pos[3 * j] - xi[0]) + (double)n0 * g.len[0];
            const double dy = (pos[3 * j + 1] - xi[1]) + (double)n1 * g.len[1];
            const double dz = (pos[3 * j + 2] - xi[2]) + (double)n2 * g.len[2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            hit = r2 < rc2 && !(j == i && n0 == 0 && n1 == 0 && n2 == 0);
            if (FILL && hit) {
              if (n0 < -127 || n0 > 127 || n1 < -127 || n1 > 127 || n2 < -127 || n2 > 127) atomicOr(err, 1);
              key = ((uint64_t)(uint32_t)j << 24) | ((uint64_t)((n0 + 128) & 255) << 16) |
                    ((uint64_t)((n1 + 128) & 255) << 8) | (uint64_t)((n2 + 128) & 255);
            }
          }
          const uint64_t mask = __ballot(hit);
          if (FILL && hit) keys[base + n_found + __popcll(mask & below)] = key;
          n_found += __popcll(mask);
        }
      }
    }
  }
  if (!FILL && lane == 0) count[i] = n_found;
}

// One wave per row: rank sort of distinct 64-bit keys (rank = number of
// smaller keys in the row), then split into src and packed shift.
__global__ void __launch_bounds__(256) k_sort_rows(const int* __restrict__ row_ptr, int N, uint64_t* __restrict__ keys,
                                                   int* __restrict__ src, int* __restrict__ shift) {
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wave >= N) return;
  const int a = row_ptr[wave], b = row_ptr[wave + 1];
  const int len = b - a;
  for (int e = lane; e < len; e += 64) {
    const uint64_t k = keys[a + e];
    int rank = 0;
    for (int f = 0; f < len; ++f) rank += keys[a + f] < k ? 1 : 0;
    src[a + rank] = (int)(k >> 24);
    shift[a + rank] = (int)(k & 0xFFFFFF);
  }
}

// keys must be rewritten in sorted order before the reverse search; done by
// rebuilding them from src/shift.
__global__ void k_rekey(const int* __restrict__ src, const int* __restrict__ shift, int E, uint64_t* __restrict__ keys) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  keys[e] = ((uint64_t)(uint32_t)src[e] << 24) | (uint64_t)(uint32_t)shift[e];
}

__global__ void k_reverse(const int* __restrict__ row_ptr, const uint64_t* __restrict__ keys, int N,
                          int* __restrict__ rev, int* __restrict__ err) {
  const int i = blockIdx.x;  // receiver
  const int a = row_ptr[i], b = row_ptr[i + 1];
  for (int e = a + threadIdx.x; e < b; e += blockDim.x) {
    const uint64_t k = keys[e];
    const int j = (int)(k >> 24);
    const int s = (int)(k & 0xFFFFFF);
    const int m0 = -unpack_n(s, 0), m1 = -unpack_n(s, 1), m2 = -unpack_n(s, 2);
    const uint64_t target = ((uint64_t)(uint32_t)i << 24) | ((uint64_t)((m0 + 128) & 255) << 16) |
                            ((uint64_t)((m1 + 128) & 255) << 8) | (uint64_t)((m2 + 128) & 255);
    int lo = row_ptr[j], hi = row_ptr[j + 1];
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (keys[mid] < target)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < row_ptr[j + 1] && keys[lo] == target) {
      rev[e] = lo;
    } else {
      rev[e] = -1;
      atomicOr(err, 2);
    }
  }
}

__global__ void k_unpack_shift(const int* __restrict__ packed, int E, int* __restrict__ shift3) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int s = packed[e];
  shift3[3 * e] = unpack_n(s, 0);
  shift3[3 * e + 1] = unpack_n(s, 1);
  shift3[3 * e + 2] = unpack_n(s, 2);
}

// d = (r_j - r_i) + n . L in FP64 (the same expression as at build time, so
// an edge and its reverse get exactly opposite vectors and equal lengths).
__device__ __forceinline__ void edge_vec(const double* __restrict__ pos, const double* __restrict__ L, int i, int j,
                                         int s, double& dx, double& dy, double& dz) {
  dx = (pos[3 * j] - pos[3 * i]) + (double)unpack_n(s, 0) * L[0];
  dy = (pos[3 * j + 1] - pos[3 * i + 1]) + (double)unpack_n(s, 1) * L[1];
  dz = (pos[3 * j + 2] - pos[3 * i + 2]) + (double)unpack_n(s, 2) * L[2];
}

__global__ void __launch_bounds__(256) k_prune_count(const double* __restrict__ pos, const int* __restrict__ owner,
                                                     const double* __restrict__ box, const int* __restrict__ row_ptr,
                                                     const int* __restrict__ src, const int* __restrict__ shift, int N,
                                                     double rc2, int* __restrict__ cnt) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const double* L = box + 3 * owner[i];
  const int a = row_ptr[i], b = row_ptr[i + 1];
  int total = 0;
  for (int base = a; base < b; base += 64) {
    const int e = base + lane;
    bool keep = false;
    if (e < b) {
      double dx, dy, dz;
      edge_vec(pos, L, i, src[e], shift[e], dx, dy, dz);
      keep = dx * dx + dy * dy + dz * dz < rc2;
    }
    total += __popcll(__ballot(keep));
  }
  if (lane == 0) cnt[i] = total;
}

__global__ void __launch_bounds__(256) k_prune_compact(const double* __restrict__ pos, const int* __restrict__ owner,
                                                       const double* __restrict__ box, const int* __restrict__ row_ptr,
                                                       const int* __restrict__ src, const int* __restrict__ shift,
                                                       const int* __restrict__ row_ptr_x, int N, double rc2,
                                                       int* __restrict__ src_x, float4* __restrict__ dvec_x,
                                                       int* __restrict__ old_idx, int* __restrict__ new_idx) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const double* L = box + 3 * owner[i];
  const int a = row_ptr[i], b = row_ptr[i + 1];
  int out = row_ptr_x[i];
  for (int base = a; base < b; base += 64) {
    const int e = base + lane;
    bool keep = false;
    double dx = 0, dy = 0, dz = 0, r2 = 0;
    int j = 0;
    if (e < b) {
      j = src[e];
      edge_vec(pos, L, i, j, shift[e], dx, dy, dz);
      r2 = dx * dx + dy * dy + dz * dz;
      keep = r2 < rc2;
    }
    const uint64_t m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (e < b) {
      if (keep) {
        const int o = out + before;
        src_x[o] = j;
        dvec_x[o] = make_float4((float)dx, (float)dy, (float)dz, (float)sqrt(r2));
        old_idx[o] = e;
        new_idx[e] = o;
      } else {
        new_idx[e] = -1;
      }
    }
    out += __popcll(m);
  }
}

// The pruned reverse index, and per receiver the number of edges that own
// their pair: e owns {e, rev(e)} when e < rev(e), or alone when its reverse
// is not listed. The two edges of a pair have exactly opposite vectors and
// equal lengths, so a function of the length is computed once per owner.
__device__ __forceinline__ bool owns_pair(int e, int re) { return re < 0 || e < re; }

__global__ void __launch_bounds__(256) k_prune_rev(const int* __restrict__ row_ptr_x, int N,
                                                   const int* __restrict__ old_idx, const int* __restrict__ new_idx,
                                                   const int* __restrict__ rev_skin, int* __restrict__ rev_x,
                                                   int* __restrict__ own_cnt) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const int a = row_ptr_x[i], b = row_ptr_x[i + 1];
  int total = 0;
  for (int base = a; base < b; base += 64) {
    const int e = base + lane;
    bool own = false;
    if (e < b) {
      const int re = new_idx[rev_skin[old_idx[e]]];
      rev_x[e] = re;
      own = owns_pair(e, re);
    }
    total += __popcll(__ballot(own));
  }
  if (lane == 0) own_cnt[i] = total;
}

// the owners in edge order, own[own_ptr[i] + k] = the k-th owner of row i,
// and each edge's pair index (its owner's position in own)
__global__ void __launch_bounds__(256) k_pair_owners(const int* __restrict__ row_ptr_x, int N,
                                                     const int* __restrict__ rev_x, const int* __restrict__ own_ptr,
                                                     int* __restrict__ own, int* __restrict__ pair_of) {
  const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= N) return;
  const int a = row_ptr_x[i], b = row_ptr_x[i + 1];
  int out = own_ptr[i];
  for (int base = a; base < b; base += 64) {
    const int e = base + lane;
    const int re = e < b ? rev_x[e] : -1;
    const bool o = e < b && owns_pair(e, re);
    const uint64_t m = __ballot(o);
    if (o) {
      const int p = out + __popcll(m & ((1ull << lane) - 1ull));
      own[p] = e;
      pair_of[e] = p;
      if (re >= 0) pair_of[re] = p;
    }
    out += __popcll(m);
  }
}

inline int blocks(long n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

void launch_owner(const int64_t* offsets, int S, int* owner, hipStream_t st) {
  k_owner<<<S, 256, 0, st>>>(offsets, owner);
}
void launch_bbox(const double* pos, const int64_t* offsets, int S, double* bbox, hipStream_t st) {
  k_bbox<<<S, 256, 0, st>>>(pos, offsets, bbox);
}
void launch_exclusive_scan(const int* in, int* out, int n, hipStream_t st) {
  k_exclusive_scan<<<1, 1024, 0, st>>>(in, out, n);
}
void launch_bin(const double* pos, const int* owner, const GridPlan* plan, int N, int* atom_cell, int* wrap,
                int* cell_count, hipStream_t st) {
  if (N == 0) return;
  k_bin<<<blocks(N, 256), 256, 0, st>>>(pos, owner, plan, N, atom_cell, wrap, cell_count);
}
void launch_bin_fill(const int* atom_cell, const int* cell_start, int N, int* cell_fill, int* cell_atoms,
                     hipStream_t st) {
  if (N == 0) return;
  k_bin_fill<<<blocks(N, 256), 256, 0, st>>>(atom_cell, cell_start, N, cell_fill, cell_atoms);
}
void launch_edges(bool fill, const double* pos, const int* owner, const GridPlan* plan, const int* atom_cell,
                  const int* wrap, const int* cell_start, const int* cell_atoms, const int* row_ptr, int N,
                  double rc2, int* count, uint64_t* keys, int* err, hipStream_t st) {
  (void)atom_cell;
  if (N == 0) return;
  if (fill)
    k_edges<true><<<blocks((long)N * 64, 256), 256, 0, st>>>(pos, owner, plan, wrap, cell_start, cell_atoms, row_ptr,
                                                              N, rc2, count, keys, err);
  else
    k_edges<false><<<blocks((long)N * 64, 256), 256, 0, st>>>(pos, owner, plan, wrap, cell_start, cell_atoms, row_ptr,
                                                               N, rc2, count, keys, err);
}
void launch_sort_rows(const int* row_ptr, int N, uint64_t* keys, int* src, int* shift, hipStream_t st) {
  if (N == 0) return;
  k_sort_rows<<<blocks((long)N * 64, 256), 256, 0, st>>>(row_ptr, N, keys, src, shift);
}
void launch_reverse(const int* row_ptr, const uint64_t* keys, int N, int* rev, int* err, hipStream_t st) {
  if (N == 0) return;
  k_reverse<<<N, 64, 0, st>>>(row_ptr, keys, N, rev, err);
}
void launch_rekey(const int* src, const int* shift, int E, uint64_t* keys, hipStream_t st) {
  if (E == 0) return;
  k_rekey<<<blocks(E, 256), 256, 0, st>>>(src, shift, E, keys);
}
void launch_unpack_shift(const int* shift_packed, int E, int* shift3, hipStream_t st) {
  if (E == 0) return;
  k_unpack_shift<<<blocks(E, 256), 256, 0, st>>>(shift_packed, E, shift3);
}
void launch_prune_count(const double* pos, const int* owner, const double* box, const int* row_ptr, const int* src,
                        const int* shift, int N, double rc2, int* cnt, hipStream_t st) {
  if (N == 0) return;
  k_prune_count<<<blocks((long)N * 64, 256), 256, 0, st>>>(pos, owner, box, row_ptr, src, shift, N, rc2, cnt);
}
void launch_prune_compact(const double* pos, const int* owner, const double* box, const int* row_ptr, const int* src,
                          const int* shift, const int* row_ptr_x, int N, double rc2, int* src_x, float4* dvec_x,
                          int* old_idx, int* new_idx, hipStream_t st) {
  if (N == 0) return;
  k_prune_compact<<<blocks((long)N * 64, 256), 256, 0, st>>>(pos, owner, box, row_ptr, src, shift, row_ptr_x, N, rc2,
                                                              src_x, dvec_x, old_idx, new_idx);
}
void launch_prune_rev(const int* row_ptr_x, int N, const int* old_idx, const int* new_idx, const int* rev_skin,
                      int* rev_x, int* own_cnt, int* own_ptr, int* own, int* pair_of, hipStream_t st) {
  if (N == 0) {
    launch_exclusive_scan(own_cnt, own_ptr, 0, st);  // own_ptr[0] = 0
    return;
  }
  k_prune_rev<<<blocks((long)N * 64, 256), 256, 0, st>>>(row_ptr_x, N, old_idx, new_idx, rev_skin, rev_x, own_cnt);
  launch_exclusive_scan(own_cnt, own_ptr, N, st);
  k_pair_owners<<<blocks((long)N * 64, 256), 256, 0, st>>>(row_ptr_x, N, rev_x, own_ptr, own, pair_of);
}

}  // namespace e3mi
