// Host-side runtime pieces shared by the library's translation units:
// error type, allocator wrapper, device buffers, and the launchers each
// kernel file exports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/e3mi.h"

namespace e3mi {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define E3MI_HIP(call)                                                                       \
  do {                                                                                       \
    hipError_t e3mi_err_ = (call);                                                           \
    if (e3mi_err_ != hipSuccess)                                                             \
      throw ::e3mi::Error(E3MI_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e3mi_err_)); \
  } while (0)

#define E3MI_REQUIRE(cond, code, msg)                  \
  do {                                                 \
    if (!(cond)) throw ::e3mi::Error((code), (msg));   \
  } while (0)

struct Allocator {
  e3mi_alloc_fn alloc = nullptr;
  e3mi_free_fn free_fn = nullptr;
  void* ctx = nullptr;
  // arena mode (arena not NULL): hand out consecutive 256-byte aligned pieces
  // of [arena, arena + arena_bytes) and never free; nothing is allocated
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  void* get(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (arena) {
      const size_t need = (bytes + 255) & ~(size_t)255;
      if (need > arena_bytes - arena_used)
        throw Error(E3MI_ENOMEM, "the evaluation needs more than the static scratch of " +
                                     std::to_string(arena_bytes) + " bytes");
      void* p = arena + arena_used;
      arena_used += need;
      return p;
    }
    void* p = nullptr;
    if (alloc) {
      p = alloc(bytes, ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
    }
    if (!p) throw Error(E3MI_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
  }
  void put(void* p) {
    if (!p || arena) return;
    if (free_fn) {
      free_fn(p, ctx);
    } else if (!alloc) {
      (void)hipFree(p);
    }
  }
};

// A device allocation that can only grow. Contents are not preserved on growth.
struct DevBuf {
  Allocator* a = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(Allocator* al) : a(al) {}
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p && a) a->put(p);
    p = nullptr;
    bytes = 0;
  }
  void* ensure(size_t n) {
    if (n > bytes || !p) {
      release();
      p = a->get(n);
      bytes = n == 0 ? 256 : n;
    }
    return p;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};


// Optional per-stage timing with HIP events recorded on the launch stream.
struct Profiler {
  struct Pending {
    int stage;
    hipEvent_t a, b;
  };
  bool on = false;
  // record only this stage (-1: every stage) and, when >= 0, only this layer
  int only_stage = -1, only_layer = -1;
  bool wants(int stage_layer) const {
    if (!on) return false;
    if (only_stage >= 0 && stage_layer / 8 != only_stage) return false;
    return only_layer < 0 || stage_layer % 8 == only_layer;
  }
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::vector<double> ms;
  std::vector<int64_t> count;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    E3MI_HIP(hipEventCreate(&e));
    return e;
  }
  void drain() {
    for (auto& p : pending) {
      E3MI_HIP(hipEventSynchronize(p.b));
      float t = 0.f;
      E3MI_HIP(hipEventElapsedTime(&t, p.a, p.b));
      if ((int)ms.size() <= p.stage) {
        ms.resize(p.stage + 1, 0.0);
        count.resize(p.stage + 1, 0);
      }
      ms[p.stage] += t;
      count[p.stage] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void reset() {
    drain();
    ms.assign(ms.size(), 0.0);
    count.assign(count.size(), 0);
  }
  ~Profiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct ProfScope {
  Profiler* p;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(Profiler* prof, int s, hipStream_t stream) : p(prof), stage(s), st(stream) {
    if (p && p->wants(stage)) {
      a = p->get();
      E3MI_HIP(hipEventRecord(a, st));
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = p->get();
      if (hipEventRecord(b, st) == hipSuccess) p->pending.push_back({stage, a, b});
    }
  }
};

// Per-structure cell-list plan (orthorhombic periodic axes or open axes).
struct GridPlan {
  double lo[3];      // grid origin: 0 on periodic axes, bounding-box minimum on open axes
  double len[3];     // box length on periodic axes
  double inv_cw[3];  // 1 / cell width
  int nb[3];         // cells per axis
  int periodic[3];
  int cell_base;     // index of the structure's first cell in the global cell array
  int pad;
};

// ---- launchers exported by graph.hip -------------------------------------
void launch_owner(const int64_t* offsets, int S, int* owner, hipStream_t st);
void launch_bbox(const double* pos, const int64_t* offsets, int S, double* bbox, hipStream_t st);
void launch_exclusive_scan(const int* in, int* out, int n, hipStream_t st);
void launch_bin(const double* pos, const int* owner, const GridPlan* plan, int N, int* atom_cell,
                int* wrap, int* cell_count, hipStream_t st);
void launch_bin_fill(const int* atom_cell, const int* cell_start, int N, int* cell_fill,
                     int* cell_atoms, hipStream_t st);
void launch_edges(bool fill, const double* pos, const int* owner, const GridPlan* plan,
                  const int* atom_cell, const int* wrap, const int* cell_start, const int* cell_atoms,
                  const int* row_ptr, int N, double rc2, int* count, uint64_t* keys, int* err,
                  hipStream_t st);
void launch_sort_rows(const int* row_ptr, int N, uint64_t* keys, int* src, int* shift, hipStream_t st);
void launch_reverse(const int* row_ptr, const uint64_t* keys, int N, int* rev, int* err, hipStream_t st);
void launch_unpack_shift(const int* shift_packed, int E, int* shift3, hipStream_t st);
void launch_prune_count(const double* pos, const int* owner, const double* box, const int* row_ptr,
                        const int* src, const int* shift, int N, double rc2, int* cnt, hipStream_t st);
void launch_prune_compact(const double* pos, const int* owner, const double* box, const int* row_ptr,
                          const int* src, const int* shift, const int* row_ptr_x, int N, double rc2,
                          int* src_x, float4* dvec_x, int* old_idx, int* new_idx, hipStream_t st);
// rev_x, the pair owners (own_cnt [N], own_ptr [N + 1], own [E]; own_ptr[N]
// is their count on the device) and each edge's pair index (pair_of [E])
void launch_prune_rev(const int* row_ptr_x, int N, const int* old_idx, const int* new_idx,
                      const int* rev_skin, int* rev_x, int* own_cnt, int* own_ptr, int* own, int* pair_of,
                      hipStream_t st);

// ---- tensor product (tp.hip) ---------------------------------------------------
struct TpArgs {
  int lmax, kind, cpt;
  const int* row_ptr;
  const int* src;
  const float4* dvec;
  const float* R;
  int r_stride;
  const float* h;
  int h_nc;
  float* A;
  const float* dA;
  float* dR;
  float* dY;
  float* dh;
  int dh_nc;
  int dh_acc;  // node adjoint: components below dh_acc are accumulated, the rest written (<= 0: all accumulated)
  int N, C;
  float inv_nu;
  // second-order (parameter-gradient) passes
  const float4* dd;  // per-edge tangent (d_dot, r_dot)
  const float* Rd;   // tangent of R, same layout as R
  const float* hd;   // tangent of h (NULL: zero)
  float* Ad;         // out: tangent of A
  const float* Ab;   // adjoint of A
  const float* Ac;   // adjoint of the tangent of A
  float* Rb;         // out: adjoint of R
  float* Rc;         // out: adjoint of the tangent of R
  float* hb;         // in/out (+=): adjoint of h
  float* hc;         // in/out (+=): adjoint of the tangent of h (NULL: not needed)
  float* Yb;         // out: adjoint of the harmonics per edge [E, 16]
  float* Yc;         // out: adjoint of the harmonics' tangent per edge [E, 16]
  // receiver chunk (first-order kernels 0-2): receivers i0 .. i0 + n_recv - 1
  // (n_recv 0: all N from i0 = 0), R and dR indexed from edge e_first
  int i0, n_recv, e_first;
  const int* rev;  // reverse edge of each edge (-1: pruned), for the sender-side adjoint and pass 7
  float* msg;      // per-edge sender-gradient messages [edges of the chunk, NIN, C] (passes 1 and 7), or NULL
  int r_bf16;      // R and dR stored as BF16 (passes 0 and 1, and the sender-side adjoint)
  int* touched;    // with msg: per atom, set to `tag` for every sender of the chunk's edges (pass 1), read by pass 7
  int tag;
  // R rows per edge pair (passes 0-2 and the sender-side adjoint): edge e's
  // weights in row r_row[e] (NULL: row e - e_first); dR stays per edge
  const int* r_row;
};
// which: 0 forward, 1 edge adjoint (dR, dY), 2 node adjoint (dh += ...),
//        3 tangent forward (Ad), 4 second-order edge adjoint (Rb, Rc),
//        5 second-order node adjoint (hb, hc += ...),
//        6 adjoints of the harmonics and their tangent (Yb, Yc) for Hessian-vector products,
//        7 node adjoint from the messages that pass 1 wrote (msg set), for the
//          chunk's receivers [i0, i0 + n_recv) as senders' partners
void launch_tp(int which, const TpArgs& a, hipStream_t st);
// scalar-output layer with R of every edge in memory (tps.hip): the
// sender-side adjoint, dR and dY of pass 1 and, when a.dh is set, dh of pass 2
bool tps_supported(const TpArgs& a);
void launch_tps_sender(const TpArgs& a, hipStream_t st);

// ---- per-atom stages (node.hip) -----------------------------------------------------
// Rows of a matrix whose row r lives at base + (r / g) * s_atom + (r % g) * s_m
// (an atom block of g = 2l + 1 rows); the row itself is contiguous.
struct RowMap {
  float* base;
  long s_atom;
  long s_m;
  int g;
};
// C[M x Nc] (+)= A0[M x k0] B0[k0 x Nc] + A1[M x k1] B1[k1 x Nc]; B row-major.
struct GemmArgs {
  RowMap a0;
  const float* b0;
  int ldb0, k0;
  RowMap a1;  // optional second product (k1 = 0: none)
  const float* b1;
  int ldb1, k1;
  RowMap c;
  int M, Nc, accumulate;
};
void launch_gemm(const GemmArgs& a, hipStream_t st, bool bf16 = false);
// Up to kMaxGemmGroup independent products (no output read or written by
// another of the group) in one launch. With l_max <= 3 a layer's groups hold
// at most 4 + 4 products (one per output order, plus the self connection's).
constexpr int kMaxGemmGroup = 8;
void launch_gemm_group(const GemmArgs* a, int n, hipStream_t st, bool bf16 = false);
void launch_gate_fwd(const float* ht, float* h, int N, int nc, int C, hipStream_t st);
void launch_gate_bwd(const float* ht, const float* dh, float* dht, int N, int nc, int C, hipStream_t st);
// h~ [N, C] = sum of n_parts partial products [n_parts, N, C] in order; h = silu(h~)
void launch_gate_fwd_sum(const float* part, int n_parts, float* ht, float* h, int N, int C, hipStream_t st);
void launch_embed(const int* species, const float* emb, float* h0, int N, int C, hipStream_t st);
void launch_readout(const float* h, int nc, const int* species, const float* Wr, const float* w2, const float* e0,
                    int N, int C, double* e_atom, float* dh, hipStream_t st, const float* wq = nullptr,
                    const float* bq = nullptr, float* q_raw = nullptr);
// Readout of a scalar-only last layer from its pre-gate values (the sum of
// n_parts partial products [n_parts, N, C], or h~ [N, C] when n_parts is 0),
// the gate and its adjoint folded in: writes E_i and dE/dh~ [N, C]
void launch_readout_gated(const float* xt, int n_parts, const int* species, const float* Wr, const float* w2,
                          const float* e0, int N, int C, double* e_atom, float* dht, hipStream_t st);
void launch_energy(const double* e_atom, const int64_t* off, int S, double* energy, hipStream_t st);
void launch_forces(const int* row_ptr, const int* rev, const float4* g, int N, float* F, hipStream_t st,
                   const float* extra = nullptr);

// Hessian-vector products (grad.hip): per-edge position adjoint of the
// second-order scalar through one layer's edge geometry, g (+)= ...
void launch_hvp_geo(int lmax, const int* row_ptr_x, int N, long e_cap, const float4* dvec, const float4* dd,
                    const float* Yb, const float* Yc, const float* P1g, const float* W1, float rc, int p,
                    int accumulate, float4* g, hipStream_t st);

// ---- product block of body order 2 (product.hip) -------------------------------------
struct ProductArgs {
  int lmax = 0, lout = 0, N = 0, C = 0;
  const float* at = nullptr;       // A~ [N, (lmax+1)^2, C]
  const int* species = nullptr;    // [N]
  const float* w1 = nullptr;       // [S, lout+1, C]
  const float* w2 = nullptr;       // [S, pairs, C]
  float* B = nullptr;              // forward output [N, (lout+1)^2, C]
  const float* dB = nullptr;       // adjoint input  [N, (lout+1)^2, C]
  float* dat = nullptr;            // adjoint output [N, (lmax+1)^2, C] (overwritten)
  // second-order pass: tangent A~_dot and B_dot, adjoints of B and B_dot, of
  // A~ and A~_dot, and (optional) per-atom weight-gradient rows
  const float* atd = nullptr;      // [N, (lmax+1)^2, C]
  float* Bd = nullptr;             // [N, (lout+1)^2, C] (overwritten)
  const float* Bb = nullptr;       // [N, (lout+1)^2, C]
  const float* Bc = nullptr;       // [N, (lout+1)^2, C]
  float* atb = nullptr;            // [N, (lmax+1)^2, C] (overwritten)
  float* atc = nullptr;            // [N, (lmax+1)^2, C] (overwritten)
  float* dw = nullptr;             // [N, lout+1+pairs, C]: d/dw1 then d/dw2 of atom i (overwritten)
};
int product_pair_count(int lmax, int lout);
void launch_product(bool fwd, const ProductArgs& p, hipStream_t st);
void launch_product_jvp(const ProductArgs& p, hipStream_t st);
void launch_product_dual_bwd(const ProductArgs& p, hipStream_t st);

// ---- electrostatics of open structures (coulomb.hip) ---------------------------------
// q~ = q - (sum_s q - Q_s) / N_s per structure
void launch_charge_fix(const float* q_raw, const int64_t* off, const double* Q, int S, float* q, hipStream_t st);
// soft-core Coulomb over all pairs of each structure: e_atom += 1/2 k q~_i phi_i,
// pot = k phi, fc = Coulomb forces [N, 3]; tiles = (structure, first receiver) per 64 receivers;
// waves (1, 2, 4, 8, 16) split each tile's senders
void launch_coulomb(const int2* tiles, int n_tiles, int waves, const int64_t* off, const double* pos, const float* q,
                    float r0, double* e_atom, float* pot, float* fc, hipStream_t st);
// dh[i, k] += (pot_i - mean_s pot) wq[k]; mean: scratch [S]; owner: structure of each atom
void launch_coulomb_dq(const int64_t* off, const int* owner, int S, int N, const float* pot, float* mean,
                       const float* wq, int C, float* dh, hipStream_t st);

// ---- radial MLP (radial.hip) ---------------------------------------------------------
// R (dR) is FP32, or BF16 when r_bf16 is set
// BF16 copies of a layer's radial weights (rounded to nearest even), laid out
// for the BF16 matrix-core steps: W2^T and W2 [64][64], W3^T [PC][64] and W3
// (used columns) in slabs of 32 columns, [PC / 32][64][32]. Needed when bf16
// is set.
struct RadialBf16 {
  const __bf16* W2T = nullptr;
  const __bf16* W2 = nullptr;
  const __bf16* W3T = nullptr;
  const __bf16* W3u = nullptr;
};
// The pair owners of the pruned list (own [P], P = *n_own on the device) and
// its reverse index: given, the radial MLP and its adjoint run once per edge
// pair (whole edge list only). The forward pass writes R to both edges' rows,
// or with `compact` once per pair, at row p for the owner own[p] (consumers
// then find edge e's row through the pair index).
struct EdgePairs {
  const int* own = nullptr;
  const int* n_own = nullptr;
  const int* rev = nullptr;
  int compact = 0;
};
void launch_radial_fwd(int n_basis, const float4* dvec, const int* row_ptr_x, int N, long e_cap, const float* W1,
                       const float* W2, const float* W3, int ld3, int PC, void* R, bool r_bf16, float rc, int p,
                       bool bf16, hipStream_t st, int e_first = 0, int e_end = -1, const RadialBf16* wb = nullptr,
                       const EdgePairs* pairs = nullptr);
void launch_radial_bwd(int n_basis, int lmax, const float4* dvec, const int* row_ptr_x, int N, long e_cap,
                       const float* W1, const float* W2, const float* W2T, const float* W3T, int PC, const void* dR,
                       bool r_bf16, const float* dY, float4* g, int accumulate, float rc, int p, bool bf16,
                       hipStream_t st, int e_first = 0, int e_end = -1, const RadialBf16* wb = nullptr,
                       const EdgePairs* pairs = nullptr);

// ---- second-order passes (radial.hip, grad.hip) -------------------------------------
void launch_radial_dual_fwd(int n_basis, const float4* dvec, const float4* dd, const int* row_ptr_x, int N, long e_cap,
                            const float* W1, const float* W2, const float* W3, int ld3, int PC, float* Rd, float* Bd,
                            float* P1d, float* H1d, float* P2d, float* H2d, float rc, int p, hipStream_t st);
void launch_radial_dual_bwd(const int* row_ptr_x, int N, long e_cap, const float* W2T, const float* W3T, int PC,
                            const float* Rb, const float* Rc, const float* P1d, const float* P2d, float* P1g,
                            float* P2g, hipStream_t st);
void launch_edge_tangent(const int* row_ptr, const int* src, const float4* dvec, const float* v, int N, float4* dd,
                         hipStream_t st);
void launch_gate_dual_fwd(const float* x, const float* xd, float* hd, int N, int nc, int C, hipStream_t st);
void launch_gate_dual_bwd(const float* x, const float* xd, const float* hb, const float* hc, float* xb, float* xc,
                          int N, int nc, int C, hipStream_t st);
void launch_readout_dual(const float* h, const float* hd, int nc, const int* owner, const double* gE, const float* Wr,
                         const float* w2, int N, int C, float* Pb, float* Pc, float* w2c, float* hb, float* hc,
                         float* eb, hipStream_t st);
void launch_group_sum(const float* X, long ld, const int* species, int n_groups, int N, int ncols, double* out,
                      long ld_out, hipStream_t st);
int tn_chunks(long rows);
void launch_gemm_tn(RowMap x1, RowMap y1, RowMap x2, RowMap y2, long rows, const int* rows_dev, int mo, int no,
                    float* partial, double* out, long ld_out, hipStream_t st);

// ---- species-factorised first layer (first.hip) ---------------------------------------
size_t first_lds_bytes(int l3max, int S64);
// P2 = silu(B W1) W2 [rows, 64] of the first layer: per pair owner (own, P =
// *n_own on the device) or per edge (own and n_own NULL); e_cap bounds the rows
void launch_first_hidden(const float4* dvec, const int* row_ptr_x, int N, long e_cap, const int* own,
                         const int* n_own, const float* W1, const float* W2, float rc, int p, float* P2,
                         hipStream_t st);
// forward (G) or adjoint (g) of the factorised first layer; edge e's P2 row is
// pair_of[e] (or e when pair_of is NULL)
void launch_first(bool fwd, int lmax, int l3max, const int* row_ptr, const int* src, const float4* dvec,
                  const int* species, int N, int S64, const float* W1, const float* W2T, const int* pair_of,
                  const float* P2, float* G, const float* dG, float4* g, int accumulate, float rc, int p,
                  hipStream_t st);

// ---- fused last layer (last.hip) ----------------------------------------------------------
struct LastArgs {
  int lmax, C, N;
  const int* row_ptr;
  const int* src;
  const float4* dvec;
  const float* h;    // layer input [N, (lmax+1)^2, C]
  const float* W1;   // [8, 64]
  const float* W2;   // [64, 64]
  const float* W2T;  // [64, 64]
  const float* W3;   // [64, ldw3], scalar-output paths in the first (lmax+1) C columns
  int ldw3;
  const float* W3T;  // [(lmax+1) C, 64]
  float* A;          // forward out: [N, lmax+1, C], nu^-1 applied
  const float* dA;   // adjoint in: [N, lmax+1, C] (without nu^-1)
  float4* g;         // adjoint out: per-edge dE/dd (+= when accumulate)
  int accumulate;
  float* dh;         // adjoint out (+=): [N, (lmax+1)^2, C]
  float rc, inv_nu;
  int p;
};
bool last_supported(int lmax, int C);
void launch_last(bool fwd, const LastArgs& a, hipStream_t st);

// ---- MD (md.hip) -----------------------------------------------------------------------
void launch_kick(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa, int N,
                 hipStream_t st);
// the drifts raise *flag to `stamp` when an atom is more than sqrt(limit2) from
// x_ref, and (probe not NULL) raise *probe to the bits of the largest
// |x - x_ref| + dt_next |v| over the atoms
void launch_drift(double* x, const double* v, const double* x_ref, double dt, double limit2, int N,
                  unsigned long long* flag, unsigned long long stamp, unsigned long long* probe, double dt_next,
                  hipStream_t st);
// k_kick then k_drift in one pass (same arithmetic)
void launch_kick_drift(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa,
                       double* x, const double* x_ref, double dt, double limit2, int N, unsigned long long* flag,
                       unsigned long long stamp, unsigned long long* probe, double dt_next, hipStream_t st);
// k_kick, with the n_copy structure energies copied e_src -> e_dst in the same
// launch; v_prev (may be NULL) receives the velocities before the kick;
// probe_clear (may be NULL) is set to 0
void launch_kick_copy(double* v, const float* F, const int* species, const double* inv_mass, double half_dt_kappa,
                      int N, const double* e_src, double* e_dst, int n_copy, double* v_prev,
                      unsigned long long* probe_clear, hipStream_t st);
void launch_nonfinite(const double* x, int n, int* flag, hipStream_t st);
// zero `bytes` (a multiple of 4) at p with a kernel (no memset node in a captured graph)
void launch_zero(void* p, size_t bytes, hipStream_t st);
void launch_species_range(const int* species, int n, int n_species, int* flag, hipStream_t st);
void launch_scale_positions(double* x, const int* owner, const double* lam, int N, hipStream_t st);
void launch_restore_rows(double* x, const double* x_save, const int* owner, const int* keep, int N, hipStream_t st);
void launch_ou(double* v, const int* species, const double* inv_mass, const int* owner, const int64_t* offsets,
               const uint64_t* seeds, const int64_t* step0, int64_t step, double c1, double c2, double kT_kappa, int N,
               hipStream_t st);
void launch_rekey(const int* src, const int* shift, int E, uint64_t* keys, hipStream_t st);

}  // namespace e3mi
