// Host runtime and C ABI of the e3mi library (declared in include/e3mi.h).
//
// Owns the model (FP32 device copies of the weights, plus transposed copies
// the adjoint GEMMs read), the neighbour-list handles and the MD state, and
// sequences the kernels of one energy + forces evaluation on the caller's
// stream:
//   prune -> embed -> for each layer: radial MLP, tensor product + neighbour
//   sum, channel mix, gate -> readout -> FP64 energy sum
//   -> adjoint in reverse layer order -> force assembly.
// The last layer keeps only its scalar outputs (the readout reads nothing
// else), which removes its l3 > 0 paths without changing E or F.
#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "cg_tables.inc"
#include "common.h"
#include "runtime.h"

namespace e3mi {

namespace {

thread_local std::string g_last_error;

// ---- configuration ---------------------------------------------------------------
struct Config {
  int lmax = 0, channels = 0, layers = 0, n_species = 0, n_basis = 0, envelope_p = 0, radial_hidden = 0,
      readout_hidden = 0;
  double cutoff = 0, avg_neighbors = 0;
  // Section 5.1 electrostatics: charge head + soft-core Coulomb (open structures)
  bool coulomb = false;
  double soft_core_r0 = 0;
  // 2: a product block of body order 2 (MACE's symmetric contraction) in every layer
  int correlation = 1;
};

size_t json_find(const std::string& s, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) return p;
  p = s.find(':', p + k.size());
  if (p == std::string::npos) throw Error(E3MI_EINVAL, std::string("config: malformed value of ") + key);
  p = s.find_first_not_of(" \t\r\n", p + 1);
  if (p == std::string::npos) throw Error(E3MI_EINVAL, std::string("config: malformed value of ") + key);
  return p;
}

// An optional JSON boolean (absent: false).
bool json_bool(const std::string& s, const char* key) {
  const size_t p = json_find(s, key);
  if (p == std::string::npos) return false;
  if (s.compare(p, 4, "true") == 0) return true;
  if (s.compare(p, 5, "false") == 0) return false;
  throw Error(E3MI_EINVAL, std::string("config: value of ") + key + " is not true or false");
}

double json_number(const std::string& s, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) throw Error(E3MI_EINVAL, std::string("config: missing key ") + key);
  p = s.find(':', p + k.size());
  if (p == std::string::npos) throw Error(E3MI_EINVAL, std::string("config: malformed value of ") + key);
  const char* b = s.c_str() + p + 1;
  char* e = nullptr;
  const double v = std::strtod(b, &e);
  if (e == b) throw Error(E3MI_EINVAL, std::string("config: value of ") + key + " is not a number");
  return v;
}

Config parse_config(const char* json) {
  E3MI_REQUIRE(json, E3MI_EINVAL, "config is NULL");
  const std::string s(json);
  Config c;
  c.lmax = (int)json_number(s, "lmax");
  c.channels = (int)json_number(s, "channels");
  c.layers = (int)json_number(s, "layers");
  c.n_species = (int)json_number(s, "n_species");
  c.cutoff = json_number(s, "cutoff");
  c.avg_neighbors = json_number(s, "avg_neighbors");
  c.n_basis = (int)json_number(s, "n_basis");
  c.envelope_p = (int)json_number(s, "envelope_p");
  c.radial_hidden = (int)json_number(s, "radial_hidden");
  c.readout_hidden = (int)json_number(s, "readout_hidden");
  c.coulomb = json_bool(s, "coulomb");
  c.correlation = json_find(s, "correlation") == std::string::npos ? 1 : (int)json_number(s, "correlation");
  E3MI_REQUIRE(c.correlation == 1 || c.correlation == 2, E3MI_EUNSUPPORTED, "correlation must be 1 or 2");
  if (c.coulomb) {
    c.soft_core_r0 = json_number(s, "soft_core_r0");
    E3MI_REQUIRE(c.soft_core_r0 > 0 && std::isfinite(c.soft_core_r0), E3MI_EINVAL, "soft_core_r0 must be positive");
  }
  E3MI_REQUIRE(c.lmax == 2 || c.lmax == 3, E3MI_EUNSUPPORTED, "lmax must be 2 or 3");
  E3MI_REQUIRE(c.channels == 32 || c.channels == 64 || c.channels == 128, E3MI_EUNSUPPORTED,
               "channels must be 32, 64 or 128");
  E3MI_REQUIRE(c.layers >= 1 && c.layers <= 8, E3MI_EINVAL, "layers must be in [1, 8]");
  E3MI_REQUIRE(c.n_species >= 1, E3MI_EINVAL, "n_species must be >= 1");
  E3MI_REQUIRE(c.cutoff > 0 && std::isfinite(c.cutoff), E3MI_EINVAL, "cutoff must be positive");
  E3MI_REQUIRE(c.avg_neighbors > 0, E3MI_EINVAL, "avg_neighbors must be positive");
  E3MI_REQUIRE(c.n_basis == 8, E3MI_EUNSUPPORTED, "n_basis must be 8");
  E3MI_REQUIRE(c.envelope_p >= 2 && c.envelope_p <= 16, E3MI_EINVAL, "envelope_p must be in [2, 16]");
  E3MI_REQUIRE(c.radial_hidden == 64, E3MI_EUNSUPPORTED, "radial_hidden must be 64");
  E3MI_REQUIRE(c.readout_hidden == 16, E3MI_EUNSUPPORTED, "readout_hidden must be 16");
  return c;
}

// Path bookkeeping of layer t (1-based).
struct LayerPlan {
  int kind;
  int l1max;           // highest input order
  int l3max_used;      // highest order of the neighbour sum A (and its mix A~) computed
  int lout;            // highest order of h~^t (0 for the last layer)
  int nc_in, nc_out;   // components of h^{t-1} and of h~^t as stored
  int nc_a;            // components of A~ = (l3max_used + 1)^2
  int n_prod;          // couplings of the product block (0 without it)
  int p_full;          // paths in the weight tensors of this layer
  int p_full_l3[4];    // per output order
  int p_used;          // paths evaluated
  int p_used_l3[4];
  long a_per_atom;     // floats of A per atom = sum_l3 (2 l3 + 1) P_l3 C
};

LayerPlan plan_layer(const Config& c, int t) {
  LayerPlan L{};
  const int T = c.layers;
  // with the product block every order of A~ feeds the products, so even the
  // last layer computes all orders of A (its outputs stay scalar)
  const bool prod = c.correlation == 2;
  L.kind = prod ? (t == 1 ? 0 : 1) : (T == 1 ? 3 : (t == 1 ? 0 : (t == T ? 2 : 1)));
  L.l1max = t == 1 ? 0 : c.lmax;
  L.l3max_used = (prod || t < T) ? c.lmax : 0;
  L.lout = t == T ? 0 : c.lmax;
  L.nc_in = (L.l1max + 1) * (L.l1max + 1);
  L.nc_out = (L.lout + 1) * (L.lout + 1);
  L.nc_a = (L.l3max_used + 1) * (L.l3max_used + 1);
  L.n_prod = prod ? product_pair_count(c.lmax, L.lout) : 0;
  for (int l = 0; l < 4; ++l) L.p_full_l3[l] = L.p_used_l3[l] = 0;
  for (int g = 0; g < e3mi_cg::kNumPaths; ++g) {
    const int l1 = e3mi_cg::kL1[g], l2 = e3mi_cg::kL2[g], l3 = e3mi_cg::kL3[g];
    if (l1 > L.l1max || l2 > c.lmax || l3 > c.lmax) continue;
    L.p_full_l3[l3]++;
    if (l3 <= L.l3max_used) L.p_used_l3[l3]++;
  }
  L.p_full = L.p_used = 0;
  L.a_per_atom = 0;
  for (int l = 0; l <= c.lmax; ++l) {
    L.p_full += L.p_full_l3[l];
    L.p_used += L.p_used_l3[l];
    L.a_per_atom += (long)(2 * l + 1) * L.p_used_l3[l] * c.channels;
  }
  return L;
}

size_t weight_count(const Config& c) {
  const size_t C = c.channels, H = c.radial_hidden;
  size_t n = (size_t)c.n_species * C;
  for (int t = 1; t <= c.layers; ++t) {
    const LayerPlan L = plan_layer(c, t);
    n += (size_t)c.n_basis * H + H * H + H * (size_t)L.p_full * C;
    for (int l = 0; l <= c.lmax; ++l) n += (size_t)L.p_full_l3[l] * C * C;
    n += (size_t)(L.l1max + 1) * C * C;  // self connection per input order
    if (L.n_prod)  // product block: w1, w2 and the linear after it
      n += (size_t)c.n_species * (L.lout + 1) * C + (size_t)c.n_species * L.n_prod * C + (L.lout + 1) * C * C;
  }
  n += C * c.readout_hidden + c.readout_hidden + c.n_species;
  if (c.coulomb) n += C + c.n_species;  // charge head and per-species charge offset
  return n;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Timed stages (per layer where it applies: index = stage * 8 + layer).
enum Stage : int {
  kPrune = 0, kEmbed, kRadialFwd, kTpFwd, kMixFwd, kGateFwd, kReadout, kGateBwd, kMixBwd, kTpBwdEdge,
  kRadialBwd, kTpBwdNode, kForces, kMdUpdate, kGraphBuild, kFirstFwd, kFirstBwd, kLastFwd, kLastBwd, kBarostat, kCoulomb, kProductFwd, kProductBwd,
  kNumStages
};
const char* const kStageNames[kNumStages] = {
    "prune", "embed", "radial_fwd", "tp_fwd", "mix_fwd", "gate_fwd", "readout", "gate_bwd", "mix_bwd",
    "tp_bwd_edge", "radial_bwd", "tp_bwd_node", "forces", "md_update", "graph_build", "first_fwd", "first_bwd",
    "last_fwd", "last_bwd", "barostat", "coulomb", "product_fwd", "product_bwd"};
inline int stage_id(Stage s, int layer = 0) { return (int)s * 8 + layer; }

}  // namespace

// ---- model -----------------------------------------------------------------------
struct LayerWeights {
  DevBuf rad1, rad2, rad2T, rad3, rad3T, rad3u;
  DevBuf rad2b, rad2Tb, rad3Tb, rad3ub;  // BF16 copies for the BF16 mode (see RadialBf16)
  RadialBf16 bf16_view() const {
    return RadialBf16{rad2Tb.as<__bf16>(), rad2b.as<__bf16>(), rad3Tb.as<__bf16>(), rad3ub.as<__bf16>()};
  }
  DevBuf mix[4], mixT[4], self_[4], selfT[4];
  DevBuf sym1, sym2, lin[4], linT[4];  // product block
};

struct Workspace {
  std::vector<std::unique_ptr<DevBuf>> h, ht, R;
  std::unique_ptr<DevBuf> A, dR, dY, g, dh_a, dh_b, dht, e_atom;
  // second-order pass: per layer A, tangents and stored radial activations
  std::vector<std::unique_ptr<DevBuf>> Al, Ad, hd, htd, Rd, P1d, H1d, P2d, H2d;
  std::unique_ptr<DevBuf> dd, Bd, Prb, Prc, w2c, eb, xb, xc, Ab, Ac, hb_a, hb_b, hc_a, hc_b, Rb, Rc, P1g, P2g,
      partial, vf;
  std::unique_ptr<DevBuf> G1, dG1;  // first layer, [N, (l3+1)^2, S*64]
  std::unique_ptr<DevBuf> P2f;      // first layer's second hidden pre-activation per edge pair (or edge), [., 64]
  std::unique_ptr<DevBuf> q_raw, q, pot, fc, pot_mean;  // electrostatics: charges, potential, forces
  std::vector<std::unique_ptr<DevBuf>> at;             // product block: A~ per layer
  std::unique_ptr<DevBuf> Ygb, Ygc, ghv, zeroE;        // Hessian-vector products
  std::vector<int> rp_host;                            // pruned row pointer on the host (receiver chunks)
  bool rp_valid = false;
  std::unique_ptr<DevBuf> Bp, dat;                     // product block: B (or dB), dA~
  // product block, second-order pass: A~_dot and B_dot per layer; adjoints of
  // B, B_dot, A~, A~_dot; per-atom weight-gradient rows
  std::vector<std::unique_ptr<DevBuf>> atd, Bpd;
  std::unique_ptr<DevBuf> Bpb, Bpc, atb, atc, dwp;
  std::unique_ptr<DevBuf> mixp;                        // partial products of a K-split channel mix
  std::unique_ptr<DevBuf> msg;                         // per-edge sender-gradient messages of a full layer
  std::unique_ptr<DevBuf> touched;                     // per atom: tag of the last chunk that sent it a message
  unsigned msg_tag = 0;
  int last_parts = -1;  // last layer left before its gate: partial products in mixp (0: h~ in ht[T])
  bool r_bf16 = false;  // the last forward pass stored R and dR in BF16 where r_bf16_layer says so
  // per layer: evaluated in receiver chunks with R of every edge kept (the
  // adjoint reads chunk c's R at its first edge instead of recomputing it)
  std::vector<char> r_whole;
  // per layer: R stored once per edge pair (row = the edge's pair index)
  std::vector<char> r_compact;
};

}  // namespace e3mi

struct e3mi_model {
  e3mi::Config cfg;
  int precision = 0;
  e3mi::Allocator alloc;
  std::vector<e3mi::LayerPlan> plans;
  std::vector<std::unique_ptr<e3mi::LayerWeights>> lw;
  std::unique_ptr<e3mi::DevBuf> emb, read1, read2, e0, qhead, qbias;
  // first layer factorised by species: U_l [S*64, C] and U_l^T [C, S*64] per output order
  bool first_factorised = true;
  bool last_fused = false;  // per-edge last layer by default (faster here); flag 4 selects the fused one
  bool edge_pairs = true;   // radial MLP and its adjoint once per edge pair (single-chunk layers); flag 8 clears
  size_t r_chunk_bytes = size_t(8) << 30;  // most bytes of per-edge R (and dR) held at once
  // most bytes of per-edge R kept whole, summed over the layers that run in
  // receiver chunks: such a layer's adjoint then reads R instead of recomputing it
  size_t r_keep_bytes = size_t(160) << 30;
  std::unique_ptr<e3mi::DevBuf> U[4], UT[4];
  e3mi::Workspace ws;
  e3mi::Profiler prof;
};

struct e3mi_graph {
  e3mi_model* model = nullptr;
  int S = 0, N = 0;
  long E = 0;       // skin-list edges
  long E_room = 0;  // edges the edge buffers (and the models' edge workspaces) hold, >= E
  double cutoff = 0, skin = 0;
  std::vector<int64_t> off_h;
  std::vector<double> box_h;
  std::vector<uint8_t> pbc_h;
  std::unique_ptr<e3mi::DevBuf> off_d, owner, box_d, pbc_d, species, row_ptr, src, shift, rev, keys;
  std::unique_ptr<e3mi::DevBuf> cnt, row_ptr_x, src_x, dvec_x, old_idx, new_idx, rev_x, x_ref;
  // edges that own their pair {e, rev(e)} (pruned list), per receiver and in edge order
  std::unique_ptr<e3mi::DevBuf> own_cnt, own_ptr, own, pair_of;
  // electrostatics: total charge per structure, and (structure, first atom) per 64-atom tile
  std::unique_ptr<e3mi::DevBuf> charge, ctiles;
  int n_ctiles = 0, c_waves = 1;
  // cell-list scratch kept between rebuilds (grown as needed), and the grid
  // plans last uploaded (re-sent only when they change)
  std::unique_ptr<e3mi::DevBuf> bb, plan_d, cell_count, cell_start, cell_fill, cell_atoms, atom_cell, wrap, err;
  std::vector<e3mi::GridPlan> plan_h;
};

struct e3mi_md {
  e3mi_model* model = nullptr;
  e3mi_graph* graph = nullptr;
  int S = 0, N = 0;
  std::vector<int64_t> off_h;
  std::vector<double> cell_h;
  std::vector<uint8_t> pbc_h;
  double cutoff = 0, skin = 0;
  int rebuild_every = 1, since_build = 0;
  int64_t steps = 0, rebuilds = 0, skin_violations = 0;
  std::unique_ptr<e3mi::DevBuf> x, v, F, species, inv_mass, energy, flag, v_prev;
  // skin guard: the drift raises flag[0] to the stamp of a step on which an
  // atom is more than skin/2 from its position at the last build, and
  // flag[1 + stamp % 2] to its forecast of the largest displacement after the
  // next step; the host reads both through flag_host (pinned) once drift_ev
  // has passed
  unsigned long long* flag_host = nullptr;
  hipEvent_t drift_ev = nullptr;
  unsigned long long stamp = 0;
  bool rebuild_next = false;  // the forecast reached skin/2: rebuild before the next evaluation
  ~e3mi_md() {
    if (flag_host) (void)hipHostFree(flag_host);
    if (drift_ev) (void)hipEventDestroy(drift_ev);
  }
  // Langevin (BAOAB) when gamma > 0: per-structure seeds and step offsets
  double temperature = 0, gamma = 0;
  std::unique_ptr<e3mi::DevBuf> seeds, step0;
  std::vector<int64_t> step0_h;  // host copy: structure s has taken step0_h[s] + steps steps
  // Monte Carlo barostat every baro_interval steps (0: off)
  double pressure_bar = 0;
  int baro_interval = 0;
  std::vector<double> dv_max;
  std::vector<uint64_t> baro_seed;
  std::vector<int64_t> baro_move;
  int64_t baro_proposed = 0, baro_accepted = 0;
  std::unique_ptr<e3mi::DevBuf> x_save, lam, keep;
};

namespace e3mi {
namespace {

std::unique_ptr<DevBuf> upload(Allocator* a, const void* host, size_t bytes) {
  auto b = std::make_unique<DevBuf>(a);
  b->ensure(bytes);
  if (bytes) E3MI_HIP(hipMemcpy(b->p, host, bytes, hipMemcpyHostToDevice));
  return b;
}

std::unique_ptr<DevBuf> upload_f32(Allocator* a, const std::vector<float>& v) {
  return upload(a, v.data(), v.size() * sizeof(float));
}

// FP32 -> BF16 bits, rounded to nearest even (finite inputs; weights are
// checked finite on upload)
uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, sizeof(u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

std::vector<float> transpose(const std::vector<float>& m, int rows, int cols) {
  std::vector<float> t((size_t)rows * cols);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c) t[(size_t)c * rows + r] = m[(size_t)r * cols + c];
  return t;
}

DevBuf& ensure(std::unique_ptr<DevBuf>& b, Allocator* a, size_t bytes) {
  if (!b) b = std::make_unique<DevBuf>(a);
  b->ensure(bytes);
  return *b;
}

void fill_plan(const Config& c, int S, const std::vector<int64_t>& off, const double* cell, const uint8_t* pbc,
               const std::vector<double>& bbox, double rc_eff, std::vector<GridPlan>& plans, int& n_cells) {
  plans.resize(S);
  n_cells = 0;
  (void)c;
  for (int s = 0; s < S; ++s) {
    GridPlan g{};
    const long ns = off[s + 1] - off[s];
    for (int k = 0; k < 3; ++k) {
      g.periodic[k] = pbc[3 * s + k] ? 1 : 0;
      if (g.periodic[k]) {
        const double L = cell[9 * s + 4 * k];
        g.lo[k] = 0.0;
        g.len[k] = L;
        g.nb[k] = std::max(1, (int)std::floor(L / rc_eff));
        g.inv_cw[k] = g.nb[k] / L;
      } else {
        const double lo = ns ? bbox[6 * s + k] : 0.0, hi = ns ? bbox[6 * s + 3 + k] : 0.0;
        const double ext = hi - lo;
        g.lo[k] = lo;
        g.len[k] = 0.0;
        g.nb[k] = ext > 0 ? std::max(1, (int)std::floor(ext / rc_eff)) : 1;
        g.inv_cw[k] = ext > 0 ? g.nb[k] / ext : 1.0;
      }
    }
    const long cap = std::max<long>(64, 8 * ns);
    long cells = (long)g.nb[0] * g.nb[1] * g.nb[2];
    if (cells > cap) {
      const double f = std::cbrt((double)cells / (double)cap);
      for (int k = 0; k < 3; ++k) {
        const int nb = std::max(1, (int)std::floor(g.nb[k] / f));
        g.inv_cw[k] *= (double)nb / g.nb[k];
        g.nb[k] = nb;
      }
      cells = (long)g.nb[0] * g.nb[1] * g.nb[2];
    }
    g.cell_base = n_cells;
    n_cells += (int)cells;
    plans[s] = g;
  }
}

void build_lists(e3mi_graph* G, const double* pos, hipStream_t st) {
  e3mi_model* M = G->model;
  Allocator* a = &M->alloc;
  const int S = G->S, N = G->N;
  const double rc_eff = G->cutoff + G->skin;
  // bounding boxes of open axes
  std::vector<double> bbox((size_t)6 * S, 0.0);
  bool any_open = false;
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < 3; ++k) any_open |= !G->pbc_h[3 * s + k];
  if (any_open && N) {
    double* bb = ensure(G->bb, a, sizeof(double) * 6 * S).as<double>();
    launch_bbox(pos, G->off_d->as<int64_t>(), S, bb, st);
    E3MI_HIP(hipMemcpyAsync(bbox.data(), bb, sizeof(double) * 6 * S, hipMemcpyDeviceToHost, st));
    E3MI_HIP(hipStreamSynchronize(st));
  }
  std::vector<double> cell9((size_t)9 * S, 0.0);
  for (int s = 0; s < S; ++s)
    for (int k = 0; k < 3; ++k) cell9[9 * s + 4 * k] = G->box_h[3 * s + k];
  std::vector<GridPlan> plans;
  int n_cells = 0;
  fill_plan(M->cfg, S, G->off_h, cell9.data(), G->pbc_h.data(), bbox, rc_eff, plans, n_cells);
  const size_t plan_bytes = sizeof(GridPlan) * plans.size();
  if (!G->plan_d || G->plan_h.size() != plans.size() ||
      std::memcmp(G->plan_h.data(), plans.data(), plan_bytes) != 0) {
    ensure(G->plan_d, a, plan_bytes);
    if (plan_bytes) E3MI_HIP(hipMemcpy(G->plan_d->p, plans.data(), plan_bytes, hipMemcpyHostToDevice));
    G->plan_h = plans;
  }
  DevBuf& plan_d = *G->plan_d;
  DevBuf& cell_count = ensure(G->cell_count, a, sizeof(int) * (n_cells + 1));
  DevBuf& cell_start = ensure(G->cell_start, a, sizeof(int) * (n_cells + 1));
  DevBuf& cell_fill = ensure(G->cell_fill, a, sizeof(int) * (n_cells + 1));
  DevBuf& cell_atoms = ensure(G->cell_atoms, a, sizeof(int) * (N + 1));
  DevBuf& atom_cell = ensure(G->atom_cell, a, sizeof(int) * (N + 1));
  DevBuf& wrap = ensure(G->wrap, a, sizeof(int) * 3 * (N + 1));
  DevBuf& err = ensure(G->err, a, sizeof(int));
  E3MI_HIP(hipMemsetAsync(cell_count.p, 0, sizeof(int) * (n_cells + 1), st));
  E3MI_HIP(hipMemsetAsync(cell_fill.p, 0, sizeof(int) * (n_cells + 1), st));
  E3MI_HIP(hipMemsetAsync(err.p, 0, sizeof(int), st));
  launch_bin(pos, G->owner->as<int>(), plan_d.as<GridPlan>(), N, atom_cell.as<int>(), wrap.as<int>(),
             cell_count.as<int>(), st);
  launch_exclusive_scan(cell_count.as<int>(), cell_start.as<int>(), n_cells, st);
  launch_bin_fill(atom_cell.as<int>(), cell_start.as<int>(), N, cell_fill.as<int>(), cell_atoms.as<int>(), st);

  const double rc2 = rc_eff * rc_eff;
  ensure(G->cnt, a, sizeof(int) * (N + 1));
  ensure(G->row_ptr, a, sizeof(int) * (N + 1));
  launch_edges(false, pos, G->owner->as<int>(), plan_d.as<GridPlan>(), atom_cell.as<int>(), wrap.as<int>(),
               cell_start.as<int>(), cell_atoms.as<int>(), nullptr, N, rc2, G->cnt->as<int>(), nullptr,
               err.as<int>(), st);
  launch_exclusive_scan(G->cnt->as<int>(), G->row_ptr->as<int>(), N, st);
  int E = 0;
  E3MI_HIP(hipMemcpyAsync(&E, G->row_ptr->as<int>() + N, sizeof(int), hipMemcpyDeviceToHost, st));
  E3MI_HIP(hipStreamSynchronize(st));
  E3MI_REQUIRE(E >= 0, E3MI_EOVERFLOW, "edge count overflow");
  G->E = E;
  // a list that outgrows its buffers on a rebuild gets 1/8 more room, so that
  // the count's drift over a trajectory does not reallocate at every rebuild
  if (E > G->E_room) G->E_room = G->E_room == 0 ? E : E + E / 8 + 64;
  const long Er = G->E_room;
  ensure(G->keys, a, sizeof(uint64_t) * (Er + 1));
  ensure(G->src, a, sizeof(int) * (Er + 1));
  ensure(G->shift, a, sizeof(int) * (Er + 1));
  ensure(G->rev, a, sizeof(int) * (Er + 1));
  launch_edges(true, pos, G->owner->as<int>(), plan_d.as<GridPlan>(), atom_cell.as<int>(), wrap.as<int>(),
               cell_start.as<int>(), cell_atoms.as<int>(), G->row_ptr->as<int>(), N, rc2, nullptr,
               G->keys->as<uint64_t>(), err.as<int>(), st);
  launch_sort_rows(G->row_ptr->as<int>(), N, G->keys->as<uint64_t>(), G->src->as<int>(), G->shift->as<int>(), st);
  launch_rekey(G->src->as<int>(), G->shift->as<int>(), E, G->keys->as<uint64_t>(), st);
  launch_reverse(G->row_ptr->as<int>(), G->keys->as<uint64_t>(), N, G->rev->as<int>(), err.as<int>(), st);
  int errh = 0;
  E3MI_HIP(hipMemcpyAsync(&errh, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  E3MI_HIP(hipStreamSynchronize(st));
  E3MI_REQUIRE(!(errh & 1), E3MI_EOVERFLOW, "image index beyond +-127 cells: wrap positions into the cell");
  E3MI_REQUIRE(!(errh & 2), E3MI_EDEVICE, "neighbour list is not symmetric");
  // pruned-list capacity and the reference positions for the skin check
  ensure(G->row_ptr_x, a, sizeof(int) * (N + 1));
  ensure(G->src_x, a, sizeof(int) * (Er + 1));
  ensure(G->dvec_x, a, sizeof(float4) * (Er + 1));
  ensure(G->old_idx, a, sizeof(int) * (Er + 1));
  ensure(G->new_idx, a, sizeof(int) * (Er + 1));
  ensure(G->rev_x, a, sizeof(int) * (Er + 1));
  ensure(G->own_cnt, a, sizeof(int) * (N + 1));
  ensure(G->own_ptr, a, sizeof(int) * (N + 1));
  ensure(G->own, a, sizeof(int) * (Er + 1));
  ensure(G->pair_of, a, sizeof(int) * (Er + 1));
  ensure(G->x_ref, a, sizeof(double) * 3 * (N + 1));
  if (N) E3MI_HIP(hipMemcpyAsync(G->x_ref->p, pos, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st));
}

e3mi_graph* new_graph(e3mi_model* M, int S, const int64_t* off, const double* pos, const int32_t* species,
                      const double* cell, const uint8_t* pbc, double cutoff, double skin, hipStream_t st) {
  E3MI_REQUIRE(M && off && cell && pbc, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(S >= 1, E3MI_EINVAL, "n_structures must be >= 1");
  E3MI_REQUIRE(off[0] == 0, E3MI_EINVAL, "atom_offsets[0] must be 0");
  for (int s = 0; s < S; ++s) E3MI_REQUIRE(off[s + 1] >= off[s], E3MI_EINVAL, "atom_offsets must be non-decreasing");
  E3MI_REQUIRE(off[S] < (1LL << 30), E3MI_EOVERFLOW, "too many atoms");
  E3MI_REQUIRE(off[S] == 0 || (pos && species), E3MI_EINVAL, "null positions or species");
  E3MI_REQUIRE(cutoff >= M->cfg.cutoff && std::isfinite(cutoff), E3MI_EINVAL,
               "graph cutoff must be at least the model cutoff");
  E3MI_REQUIRE(skin >= 0 && std::isfinite(skin), E3MI_EINVAL, "skin must be >= 0");
  auto G = std::make_unique<e3mi_graph>();
  G->model = M;
  G->S = S;
  G->N = (int)off[S];
  G->cutoff = cutoff;
  G->skin = skin;
  G->off_h.assign(off, off + S + 1);
  G->box_h.assign((size_t)3 * S, 0.0);
  G->pbc_h.assign(pbc, pbc + 3 * S);
  for (int s = 0; s < S; ++s) {
    bool periodic = false;
    for (int k = 0; k < 3; ++k) periodic |= pbc[3 * s + k] != 0;
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) {
        const double v = cell[9 * s + 3 * r + k];
        E3MI_REQUIRE(std::isfinite(v), E3MI_EINVAL, "cell is not finite");
        if (periodic && r != k && v != 0.0)
          throw Error(E3MI_EUNSUPPORTED, "periodic cells must be orthorhombic (diagonal)");
      }
    for (int k = 0; k < 3; ++k)
      if (pbc[3 * s + k]) {
        const double L = cell[9 * s + 4 * k];
        E3MI_REQUIRE(L > 0, E3MI_EINVAL, "periodic cell length must be positive");
        G->box_h[3 * s + k] = L;
      }
  }
  Allocator* a = &M->alloc;
  G->off_d = upload(a, G->off_h.data(), sizeof(int64_t) * (S + 1));
  G->box_d = upload(a, G->box_h.data(), sizeof(double) * 3 * S);
  G->pbc_d = upload(a, G->pbc_h.data(), 3 * S);
  {
    const std::vector<double> zero((size_t)S, 0.0);
    G->charge = upload(a, zero.data(), sizeof(double) * S);
  }
  if (M->cfg.coulomb) {
    for (int s = 0; s < S * 3; ++s)
      E3MI_REQUIRE(!pbc[s], E3MI_EUNSUPPORTED, "the Coulomb term is defined for open structures only (pbc all 0)");
    std::vector<int2> tiles;
    int64_t n_max = 0;
    for (int s = 0; s < S; ++s) {
      n_max = std::max<int64_t>(n_max, off[s + 1] - off[s]);
      for (int64_t i0 = off[s]; i0 < off[s + 1]; i0 += 64) tiles.push_back(make_int2(s, (int)i0));
    }
    G->n_ctiles = (int)tiles.size();
    // enough waves per tile to cover the largest structure's senders in one round, at most 16
    while (G->c_waves < 16 && 64 * G->c_waves < n_max) G->c_waves *= 2;
    G->ctiles = upload(a, tiles.data(), sizeof(int2) * tiles.size());
  }
  G->owner = std::make_unique<DevBuf>(a);
  G->owner->ensure(sizeof(int) * (G->N + 1));
  G->species = std::make_unique<DevBuf>(a);
  G->species->ensure(sizeof(int) * (G->N + 1));
  if (G->N) E3MI_HIP(hipMemcpyAsync(G->species->p, species, sizeof(int) * G->N, hipMemcpyDeviceToDevice, st));
  launch_owner(G->off_d->as<int64_t>(), S, G->owner->as<int>(), st);
  if (G->N) {
    DevBuf flag(a);
    flag.ensure(sizeof(int));
    E3MI_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), st));
    launch_nonfinite(pos, 3 * G->N, flag.as<int>(), st);
    launch_species_range(G->species->as<int>(), G->N, M->cfg.n_species, flag.as<int>(), st);
    int fh = 0;
    E3MI_HIP(hipMemcpyAsync(&fh, flag.p, sizeof(int), hipMemcpyDeviceToHost, st));
    E3MI_HIP(hipStreamSynchronize(st));
    E3MI_REQUIRE(!(fh & 8), E3MI_EINVAL, "species outside [0, n_species)");
    E3MI_REQUIRE(!fh, E3MI_ENAN, "positions are not finite");
  }
  build_lists(G.get(), pos, st);
  return G.release();
}

// ---- energy + forces ---------------------------------------------------------------

void prune(e3mi_graph* G, const double* pos, hipStream_t st) {
  const int N = G->N;
  const double rc2 = G->model->cfg.cutoff * G->model->cfg.cutoff;
  launch_prune_count(pos, G->owner->as<int>(), G->box_d->as<double>(), G->row_ptr->as<int>(), G->src->as<int>(),
                     G->shift->as<int>(), N, rc2, G->cnt->as<int>(), st);
  launch_exclusive_scan(G->cnt->as<int>(), G->row_ptr_x->as<int>(), N, st);
  launch_prune_compact(pos, G->owner->as<int>(), G->box_d->as<double>(), G->row_ptr->as<int>(), G->src->as<int>(),
                       G->shift->as<int>(), G->row_ptr_x->as<int>(), N, rc2, G->src_x->as<int>(),
                       G->dvec_x->as<float4>(), G->old_idx->as<int>(), G->new_idx->as<int>(), st);
  launch_prune_rev(G->row_ptr_x->as<int>(), N, G->old_idx->as<int>(), G->new_idx->as<int>(), G->rev->as<int>(),
                   G->rev_x->as<int>(), G->own_cnt->as<int>(), G->own_ptr->as<int>(), G->own->as<int>(),
                   G->pair_of->as<int>(), st);
}

// Channels per thread of the tensor-product kernels (threads per receiver = C / cpt).
int cpt_for(const LayerPlan& L, int C) {
  if (L.kind == 1) return 1;
  return C <= 64 ? 1 : C / 64;
}

// h~ = sum_p A_p W_l3[p] + h_in S_l3 for every computed order l3 (rows
// (atom, m), columns channels); out has out_nc components per atom. `hin` may
// be NULL (no self connection term).
void launch_mix(e3mi_model* M, const LayerPlan& L, LayerWeights& W, const float* A, const float* hin, float* ht,
                int out_nc, int N, hipStream_t st, bool bf16 = false) {
  const int C = M->cfg.channels;
  long gbase = 0;
  GemmArgs grp[kMaxGemmGroup];
  int n = 0;
  for (int l3 = 0; l3 <= L.l3max_used; ++l3) {
    const int P3 = L.p_used_l3[l3], g = 2 * l3 + 1;
    GemmArgs& ga = grp[n++] = GemmArgs{};
    ga.a0 = RowMap{const_cast<float*>(A) + gbase, (long)g * P3 * C, (long)P3 * C, g};
    ga.b0 = W.mix[l3].as<float>();
    ga.ldb0 = C;
    ga.k0 = P3 * C;
    if (hin && l3 <= L.l1max) {
      ga.a1 = RowMap{const_cast<float*>(hin) + (long)l3 * l3 * C, (long)L.nc_in * C, (long)C, g};
      ga.b1 = W.self_[l3].as<float>();
      ga.ldb1 = C;
      ga.k1 = C;
    }
    ga.c = RowMap{ht + (long)l3 * l3 * C, (long)out_nc * C, (long)C, g};
    ga.M = N * g;
    ga.Nc = C;
    gbase += (long)N * g * P3 * C;
  }
  launch_gemm_group(grp, n, st, bf16);
}

// Channel mix of a scalar-output layer split over K into independent partial
// products of 128 K each (one grouped launch): with one scalar row per atom
// the 64 x 64 output tiles are too few to fill the GPU for small systems, and
// each workgroup then walks only its part of the K slabs. The split depends
// on K only, so an atom's result does not depend on what else is in the batch.
// Partial j goes to part + j N C; returns the number of parts written.
int mix_split_parts(int K) { return std::max(1, std::min(kMaxGemmGroup, K / 128)); }
int launch_mix_scalar_split(e3mi_model* M, const LayerPlan& L, LayerWeights& W, const float* A, const float* hin,
                            float* part, int parts, int N, hipStream_t st, bool bf16) {
  const int C = M->cfg.channels;
  const int KA = L.p_used_l3[0] * C, KS = hin ? C : 0, K = KA + KS;
  const int units = (K + 31) / 32;
  GemmArgs grp[kMaxGemmGroup];
  int n = 0;
  for (int j = 0; j < parts; ++j) {
    const int kb = std::min(K, units * j / parts * 32), ke = std::min(K, units * (j + 1) / parts * 32);
    if (kb >= ke) continue;
    GemmArgs& ga = grp[n] = GemmArgs{};
    const int a_hi = std::min(ke, KA);
    ga.a0 = RowMap{const_cast<float*>(A) + std::min(kb, KA), (long)KA, (long)KA, 1};
    ga.b0 = W.mix[0].as<float>() + (long)std::min(kb, KA) * C;
    ga.ldb0 = C;
    ga.k0 = std::max(0, a_hi - kb);
    const int s_lo = std::max(kb, KA) - KA, s_hi = ke - KA;
    if (s_hi > s_lo) {
      ga.a1 = RowMap{const_cast<float*>(hin) + s_lo, (long)L.nc_in * C, (long)C, 1};
      ga.b1 = W.self_[0].as<float>() + (long)s_lo * C;
      ga.ldb1 = C;
      ga.k1 = s_hi - s_lo;
    }
    ga.c = RowMap{part + (long)n * N * C, (long)C, (long)C, 1};
    ga.M = N;
    ga.Nc = C;
    ++n;
  }
  launch_gemm_group(grp, n, st, bf16);
  return n;
}

// After the product block: h~^L = B^L W_lin,L + h_in^L S_L for L <= lout.
void launch_lin(e3mi_model* M, const LayerPlan& L, LayerWeights& W, const float* B, const float* hin, float* ht,
                int N, hipStream_t st, bool bf16) {
  const int C = M->cfg.channels;
  GemmArgs grp[kMaxGemmGroup];
  int n = 0;
  for (int l = 0; l <= L.lout; ++l) {
    const int g = 2 * l + 1;
    GemmArgs& ga = grp[n++] = GemmArgs{};
    ga.a0 = RowMap{const_cast<float*>(B) + (long)l * l * C, (long)L.nc_out * C, (long)C, g};
    ga.b0 = W.lin[l].as<float>();
    ga.ldb0 = C;
    ga.k0 = C;
    if (hin && l <= L.l1max) {
      ga.a1 = RowMap{const_cast<float*>(hin) + (long)l * l * C, (long)L.nc_in * C, (long)C, g};
      ga.b1 = W.self_[l].as<float>();
      ga.ldb1 = C;
      ga.k1 = C;
    }
    ga.c = RowMap{ht + (long)l * l * C, (long)L.nc_out * C, (long)C, g};
    ga.M = N * g;
    ga.Nc = C;
  }
  launch_gemm_group(grp, n, st, bf16);
}

// Adjoint of launch_lin: dB^L = dh~^L W_lin,L^T and (dprev not NULL) dprev^L = dh~^L S_L^T.
void launch_lin_adjoint(e3mi_model* M, const LayerPlan& L, LayerWeights& W, const float* dht, float* dB, float* dprev,
                        int N, hipStream_t st, bool bf16) {
  const int C = M->cfg.channels;
  GemmArgs grp[kMaxGemmGroup];
  int n = 0;
  for (int l = 0; l <= L.lout; ++l) {
    const int g = 2 * l + 1;
    for (int which = 0; which < 2; ++which) {
      if (which == 1 && (!dprev || l > L.l1max)) continue;
      GemmArgs& ga = grp[n++] = GemmArgs{};
      ga.a0 = RowMap{const_cast<float*>(dht) + (long)l * l * C, (long)L.nc_out * C, (long)C, g};
      ga.b0 = which == 0 ? W.linT[l].as<float>() : W.selfT[l].as<float>();
      ga.ldb0 = C;
      ga.k0 = C;
      ga.c = which == 0 ? RowMap{dB + (long)l * l * C, (long)L.nc_out * C, (long)C, g}
                        : RowMap{dprev + (long)l * l * C, (long)L.nc_in * C, (long)C, g};
      ga.M = N * g;
      ga.Nc = C;
    }
  }
  launch_gemm_group(grp, n, st, bf16);
}

ProductArgs product_args(e3mi_model* M, e3mi_graph* G, const LayerPlan& L, LayerWeights& W, const float* at) {
  ProductArgs p;
  p.lmax = M->cfg.lmax;
  p.lout = L.lout;
  p.N = G->N;
  p.C = M->cfg.channels;
  p.at = at;
  p.species = G->species->as<int>();
  p.w1 = W.sym1.as<float>();
  p.w2 = W.sym2.as<float>();
  return p;
}

// Adjoint of the channel mix: dA = dht W^T per order, and (when dprev is not
// NULL) dprev[l3] (+)= dht[l3] S^T for the orders present in the input.
void launch_mix_adjoint(e3mi_model* M, const LayerPlan& L, LayerWeights& W, const float* dht, int dht_nc, float* dA,
                        float* dprev, int N, hipStream_t st, bool bf16 = false) {
  const int C = M->cfg.channels;
  long gbase = 0;
  GemmArgs grp[kMaxGemmGroup];
  int n = 0;
  for (int l3 = 0; l3 <= L.l3max_used; ++l3) {
    const int P3 = L.p_used_l3[l3], gg = 2 * l3 + 1;
    GemmArgs& ga = grp[n++] = GemmArgs{};
    ga.a0 = RowMap{const_cast<float*>(dht) + (long)l3 * l3 * C, (long)dht_nc * C, (long)C, gg};
    ga.b0 = W.mixT[l3].as<float>();
    ga.ldb0 = P3 * C;
    ga.k0 = C;
    ga.c = RowMap{dA + gbase, (long)gg * P3 * C, (long)P3 * C, gg};
    ga.M = N * gg;
    ga.Nc = P3 * C;
    gbase += (long)N * gg * P3 * C;
  }
  for (int l3 = 0; dprev && l3 <= std::min(L.l3max_used, L.l1max); ++l3) {
    const int gg = 2 * l3 + 1;
    GemmArgs& ga = grp[n++] = GemmArgs{};
    ga.a0 = RowMap{const_cast<float*>(dht) + (long)l3 * l3 * C, (long)dht_nc * C, (long)C, gg};
    ga.b0 = W.selfT[l3].as<float>();
    ga.ldb0 = C;
    ga.k0 = C;
    ga.c = RowMap{dprev + (long)l3 * l3 * C, (long)L.nc_in * C, (long)C, gg};
    ga.M = N * gg;
    ga.Nc = C;
  }
  launch_gemm_group(grp, n, st, bf16);
}

// Whether the energy/force path evaluates layer 1 through the species
// factorisation (first.hip): always possible for layer 1 (its input is the
// embedding) when the species x hidden width fits the kernel's LDS budget.
bool factorised_first(const e3mi_model* M) {
  const int S64 = M->cfg.n_species * M->cfg.radial_hidden;
  return M->first_factorised && S64 <= 512 && first_lds_bytes(M->plans[0].l3max_used, S64) <= 65536;
}

// Whether layer t runs through the fused last-layer kernels (last.hip): the
// scalar-output last layer of a stack of two or more, in FP32, when the
// per-layer A and R are not kept for a second-order pass.
bool fused_last(const e3mi_model* M, const LayerPlan& L, bool keep_A, bool bf16) {
  return M->last_fused && L.kind == 2 && !keep_A && !bf16 && last_supported(M->cfg.lmax, M->cfg.channels);
}

LastArgs last_args(e3mi_model* M, e3mi_graph* G, const LayerPlan& L, LayerWeights& W, const float* hin) {
  const Config& c = M->cfg;
  LastArgs la{};
  la.lmax = c.lmax;
  la.C = c.channels;
  la.N = G->N;
  la.row_ptr = G->row_ptr_x->as<int>();
  la.src = G->src_x->as<int>();
  la.dvec = G->dvec_x->as<float4>();
  la.h = hin;
  la.W1 = W.rad1.as<float>();
  la.W2 = W.rad2.as<float>();
  la.W2T = W.rad2T.as<float>();
  la.W3 = W.rad3u.as<float>();
  la.ldw3 = L.p_used * c.channels;
  la.W3T = W.rad3T.as<float>();
  la.rc = (float)c.cutoff;
  la.inv_nu = (float)(1.0 / c.avg_neighbors);
  la.p = c.envelope_p;
  return la;
}

// "name" or "name@t" -> stage id (and layer t, -1 for every layer).
int parse_stage(const char* stage, int* layer) {
  std::string name(stage);
  *layer = -1;
  const size_t at = name.find('@');
  if (at != std::string::npos) {
    *layer = std::atoi(name.c_str() + at + 1);
    name = name.substr(0, at);
    E3MI_REQUIRE(*layer >= 0 && *layer < 8, E3MI_EINVAL, "layer of a stage must be in [0, 8)");
  }
  for (int k = 0; k < kNumStages; ++k)
    if (name == kStageNames[k]) return k;
  throw Error(E3MI_EINVAL, "unknown stage " + name);
}

// Per-edge R and dR of a layer in BF16 (BF16 mode, first-order pass), except
// in layers with every path: their tensor-product kernels are bound by the
// contraction over 99 outputs, not by R traffic, and the BF16 conversions push
// their adjoint past two waves per SIMD (one wave halves its speed).
bool r_bf16_layer(const Workspace& w, const LayerPlan& L) { return w.r_bf16 && L.kind != 1; }

// Receiver chunks of a layer evaluated with per-edge R in memory: each chunk's
// edges hold at most the model's r_chunk_bytes of R (and of dR in the
// adjoint), so R never needs the whole edge set at once. One chunk
// {0, N, 0, -1} (every edge, no host synchronisation) when the whole edge
// capacity fits; otherwise the pruned row pointer is read back once per
// evaluation.
struct RChunk {
  int i0, i1;  // receivers [i0, i1)
  int e0, e1;  // edges [e0, e1); e1 = -1: all edges of all receivers
};

size_t r_chunk_edges(const e3mi_model* M, long Ecap, int PCu) {
  return std::min<size_t>((size_t)(Ecap + 1), M->r_chunk_bytes / ((size_t)PCu * sizeof(float)));
}

// The pruned row pointer on the host, read back once per evaluation.
const std::vector<int>& pruned_rows(e3mi_model* M, e3mi_graph* G, hipStream_t st) {
  Workspace& w = M->ws;
  if (!w.rp_valid) {
    w.rp_host.resize((size_t)G->N + 1);
    E3MI_HIP(hipMemcpyAsync(w.rp_host.data(), G->row_ptr_x->p, sizeof(int) * ((size_t)G->N + 1),
                            hipMemcpyDeviceToHost, st));
    E3MI_HIP(hipStreamSynchronize(st));
    w.rp_valid = true;
  }
  return w.rp_host;
}

std::vector<RChunk> r_chunks(e3mi_model* M, e3mi_graph* G, int PCu, hipStream_t st) {
  const int N = G->N;
  const size_t cap = r_chunk_edges(M, G->E, PCu);
  if (cap >= (size_t)(G->E + 1)) return {RChunk{0, N, 0, -1}};
  const std::vector<int>& rp = pruned_rows(M, G, st);
  std::vector<RChunk> out;
  for (int i0 = 0; i0 < N;) {
    int i1 = i0 + 1;  // a receiver's row always fits (its edges are few)
    while (i1 < N && (size_t)(rp[i1 + 1] - rp[i0]) <= cap) ++i1;
    E3MI_REQUIRE((size_t)(rp[i1] - rp[i0]) <= cap, E3MI_EOVERFLOW, "one receiver's edges exceed the R chunk");
    out.push_back(RChunk{i0, i1, rp[i0], rp[i1]});
    i0 = i1;
  }
  return out;
}

// R of a chunk: the buffer itself, or for a layer whose R is kept whole, the
// chunk's first edge within it
void* chunk_r(const Workspace& w, int t, void* R, const RChunk& ch, int PCu, size_t elem) {
  return w.r_whole[t] && ch.e1 >= 0 ? static_cast<char*>(R) + (size_t)ch.e0 * PCu * elem : R;
}

// The pair owners of the pruned list, used by a layer's radial passes when
// the model runs them per edge pair and the chunk is the whole edge list.
EdgePairs graph_pairs(const e3mi_graph* G, bool compact = false) {
  return EdgePairs{G->own->as<int>(), G->own_ptr->as<int>() + G->N, G->rev_x->as<int>(), compact ? 1 : 0};
}
const EdgePairs* pairs_for(const e3mi_model* M, const RChunk& ch, const EdgePairs& p) {
  return M->edge_pairs && ch.e1 < 0 ? &p : nullptr;
}
// the first layer's hidden activations: row pair_of[e] per edge pair, or row e
const int* first_pair_index(const e3mi_model* M, const e3mi_graph* G) {
  return M->edge_pairs ? G->pair_of->as<int>() : nullptr;
}
// R of a layer once per edge pair: the pair mode on a single chunk, in a
// first-order evaluation (the second-order passes read R per edge)
bool r_compact_for(const e3mi_model* M, const std::vector<RChunk>& chunks, bool keep_A) {
  return M->edge_pairs && !keep_A && chunks.size() == 1 && chunks[0].e1 < 0;
}

void set_chunk(TpArgs& ta, const RChunk& ch) {
  ta.i0 = ch.e1 < 0 ? 0 : ch.i0;
  ta.n_recv = ch.e1 < 0 ? 0 : ch.i1 - ch.i0;
  ta.e_first = ch.e1 < 0 ? 0 : ch.e0;
}

// Primal forward pass: edge selection, embedding and every layer. Leaves
// h^t, h~^t and R^t of every layer in the workspace; A in one shared buffer,
// or per layer when keep_A (the parameter-gradient pass needs them).
// defer_last_gate: a scalar-only last layer (no product block) stops at its
// pre-gate values (ht, or the partial products in mixp; their count in
// last_parts) for a readout that applies the gate itself.
void forward_pass(e3mi_model* M, e3mi_graph* G, const double* pos, bool keep_A, hipStream_t st, bool bf16,
                  bool defer_last_gate = false) {
  const Config& c = M->cfg;
  Allocator* a = &M->alloc;
  const int N = G->N, S = G->S, C = c.channels, T = c.layers;
  const long Ecap = G->E_room;  // edge capacity (>= the skin-list count)
  const int NC = (c.lmax + 1) * (c.lmax + 1);
  const float inv_nu = (float)(1.0 / c.avg_neighbors);
  const float rc = (float)c.cutoff;
  const int p_env = c.envelope_p;
  Workspace& w = M->ws;
  (void)S;
  {
    ProfScope ps(&M->prof, stage_id(kPrune), st);
    prune(G, pos, st);
  }
  w.rp_valid = false;
  const int* row_ptr = G->row_ptr_x->as<int>();
  const int* src = G->src_x->as<int>();
  const float4* dvec = G->dvec_x->as<float4>();
  const int* species = G->species->as<int>();

  // ---- workspace (grows, never shrinks) ----
  w.r_bf16 = bf16 && !keep_A;
  w.h.resize(T + 1);
  w.ht.resize(T + 1);
  w.R.resize(T + 1);
  ensure(w.h[0], a, sizeof(float) * (size_t)N * C);
  long a_max = 0;
  size_t dr_bytes = 0, kept = 0;
  w.r_whole.assign(T + 1, 0);
  w.r_compact.assign(T + 1, 0);
  for (int t = 1; t <= T; ++t) {
    const LayerPlan& L = M->plans[t - 1];
    ensure(w.h[t], a, sizeof(float) * (size_t)N * L.nc_out * C);
    ensure(w.ht[t], a, sizeof(float) * (size_t)N * L.nc_out * C);
    a_max = std::max(a_max, L.a_per_atom);
    if (t == 1 && factorised_first(M) && !keep_A) continue;
    if (fused_last(M, L, keep_A, bf16)) continue;
    // the second-order pass keeps R of every edge (skin-list capacity);
    // otherwise one chunk, or every edge inside the cutoff while the layers'
    // kept R stays within r_keep_bytes
    const size_t chunk_edges = r_chunk_edges(M, Ecap, L.p_used * C);
    const size_t r_elem = r_bf16_layer(w, L) ? 2 : 4;
    size_t r_edges = keep_A ? (size_t)(Ecap + 1) : chunk_edges;
    if (!keep_A && chunk_edges < (size_t)(Ecap + 1)) {
      // room for 1/8 more edges than this call has inside the cutoff, so
      // that the count's drift between rebuilds does not reallocate
      const size_t e_in = (size_t)pruned_rows(M, G, st)[N] + 1;
      const size_t e_room = std::min((size_t)(Ecap + 1), e_in + e_in / 8);
      const size_t all_bytes = r_elem * e_room * L.p_used * C;
      if (kept + all_bytes <= M->r_keep_bytes) {
        w.r_whole[t] = 1;
        kept += all_bytes;
        r_edges = std::max(r_edges, w.R[t] && w.R[t]->bytes >= r_elem * e_in * L.p_used * C ? e_in : e_room);
      }
    }
    ensure(w.R[t], a, r_elem * r_edges * L.p_used * C);
    dr_bytes = std::max(dr_bytes, r_elem * chunk_edges * L.p_used * C);
  }
  ensure(w.A, a, sizeof(float) * (size_t)N * a_max);
  if (keep_A) {
    w.Al.resize(T + 1);
    for (int t = 1; t <= T; ++t) ensure(w.Al[t], a, sizeof(float) * (size_t)N * M->plans[t - 1].a_per_atom);
  }
  if (dr_bytes) ensure(w.dR, a, dr_bytes);
  ensure(w.dY, a, sizeof(float) * 16 * (size_t)(Ecap + 1));
  ensure(w.g, a, sizeof(float4) * (size_t)(Ecap + 1));
  ensure(w.dh_a, a, sizeof(float) * (size_t)N * NC * C);
  ensure(w.dh_b, a, sizeof(float) * (size_t)N * NC * C);
  ensure(w.dht, a, sizeof(float) * (size_t)N * NC * C);
  ensure(w.e_atom, a, sizeof(double) * (size_t)N);
  // ---- forward ----
  {
    ProfScope ps(&M->prof, stage_id(kEmbed), st);
    launch_embed(species, M->emb->as<float>(), w.h[0]->as<float>(), N, C, st);
  }
  const bool fact = factorised_first(M) && !keep_A;
  const int S64 = c.n_species * c.radial_hidden;
  if (fact) {
    ensure(w.G1, a, sizeof(float) * (size_t)N * M->plans[0].nc_a * S64);
    ensure(w.P2f, a, sizeof(float) * (size_t)c.radial_hidden * (size_t)(Ecap + 1));
    ensure(w.dG1, a, sizeof(float) * (size_t)N * M->plans[0].nc_a * S64);
  }
  // product block: the mix writes A~ (no self connection); B follows, then
  // h~ = B W_lin + h_in S
  const bool prod = c.correlation == 2;
  if (prod) {
    w.at.resize(T + 1);
    for (int t = 1; t <= T; ++t) ensure(w.at[t], a, sizeof(float) * (size_t)N * M->plans[t - 1].nc_a * C);
    ensure(w.Bp, a, sizeof(float) * (size_t)N * NC * C);
    ensure(w.dat, a, sizeof(float) * (size_t)N * NC * C);
  }
  auto product_tail = [&](int t, const LayerPlan& L, LayerWeights& W, const float* hin, float* ht) {
    ProductArgs pa = product_args(M, G, L, W, w.at[t]->as<float>());
    pa.B = w.Bp->as<float>();
    {
      ProfScope ps(&M->prof, stage_id(kProductFwd, t), st);
      launch_product(true, pa, st);
    }
    ProfScope ps(&M->prof, stage_id(kMixFwd, t), st);
    launch_lin(M, L, W, w.Bp->as<float>(), hin, ht, N, st, bf16);
  };
  for (int t = 1; t <= T; ++t) {
    const LayerPlan& L = M->plans[t - 1];
    LayerWeights& W = *M->lw[t - 1];
    const float* hin = w.h[t - 1]->as<float>();
    if (t == 1 && fact) {
      float* G1 = w.G1->as<float>();
      {
        // the hidden layers once per edge pair (per edge with flag 8), then
        // the per-species neighbour sums read them through the pair index
        ProfScope ps(&M->prof, stage_id(kFirstFwd, 1), st);
        const EdgePairs prs = graph_pairs(G);
        launch_first_hidden(dvec, row_ptr, N, Ecap, M->edge_pairs ? prs.own : nullptr,
                            M->edge_pairs ? prs.n_own : nullptr, W.rad1.as<float>(), W.rad2.as<float>(), rc, p_env,
                            w.P2f->as<float>(), st);
        launch_first(true, c.lmax, L.l3max_used, row_ptr, src, dvec, species, N, S64, W.rad1.as<float>(), nullptr,
                     first_pair_index(M, G), w.P2f->as<float>(), G1, nullptr, nullptr, 0, rc, p_env, st);
      }
      float* ht = w.ht[1]->as<float>();
      float* mix_out = prod ? w.at[1]->as<float>() : ht;
      const int mix_nc = prod ? L.nc_a : L.nc_out;
      {
        ProfScope ps(&M->prof, stage_id(kMixFwd, 1), st);
        GemmArgs grp[kMaxGemmGroup];
        int n = 0;
        for (int l3 = 0; l3 <= L.l3max_used; ++l3) {
          const int g = 2 * l3 + 1;
          GemmArgs& ga = grp[n++] = GemmArgs{};
          ga.a0 = RowMap{G1 + (long)l3 * l3 * S64, (long)L.nc_a * S64, (long)S64, g};
          ga.b0 = M->U[l3]->as<float>();
          ga.ldb0 = C;
          ga.k0 = S64;
          if (l3 == 0 && !prod) {
            ga.a1 = RowMap{const_cast<float*>(hin), (long)C, (long)C, 1};
            ga.b1 = W.self_[0].as<float>();
            ga.ldb1 = C;
            ga.k1 = C;
          }
          ga.c = RowMap{mix_out + (long)l3 * l3 * C, (long)mix_nc * C, (long)C, g};
          ga.M = N * g;
          ga.Nc = C;
        }
        launch_gemm_group(grp, n, st, bf16);
      }
      if (prod) product_tail(1, L, W, hin, ht);
      {
        ProfScope ps(&M->prof, stage_id(kGateFwd, 1), st);
        launch_gate_fwd(ht, w.h[1]->as<float>(), N, L.nc_out, C, st);
      }
      continue;
    }
    float* A = keep_A ? w.Al[t]->as<float>() : w.A->as<float>();
    if (fused_last(M, L, keep_A, bf16)) {
      LastArgs la = last_args(M, G, L, W, hin);
      la.A = A;
      {
        ProfScope ps(&M->prof, stage_id(kLastFwd, t), st);
        launch_last(true, la, st);
      }
      float* ht = w.ht[t]->as<float>();
      {
        ProfScope ps(&M->prof, stage_id(kMixFwd, t), st);
        launch_mix(M, L, W, A, hin, ht, L.nc_out, N, st, bf16);
      }
      if (defer_last_gate && t == T && L.nc_out == 1) {
        w.last_parts = 0;
        continue;
      }
      {
        ProfScope ps(&M->prof, stage_id(kGateFwd, t), st);
        launch_gate_fwd(ht, w.h[t]->as<float>(), N, L.nc_out, C, st);
      }
      continue;
    }
    float* R = w.R[t]->as<float>();  // BF16 values when r_bf16
    const int PCu = L.p_used * C;
    const std::vector<RChunk> chunks = keep_A ? std::vector<RChunk>{RChunk{0, N, 0, -1}} : r_chunks(M, G, PCu, st);
    TpArgs ta{};
    const bool lr_bf16 = r_bf16_layer(w, L);
    ta.r_bf16 = lr_bf16 ? 1 : 0;
    ta.lmax = c.lmax;
    ta.kind = L.kind;
    ta.cpt = cpt_for(L, C);
    ta.row_ptr = row_ptr;
    ta.src = src;
    ta.dvec = dvec;
    ta.R = R;
    ta.r_stride = PCu;
    ta.h = hin;
    ta.h_nc = L.nc_in;
    ta.A = A;
    ta.N = N;
    ta.C = C;
    ta.inv_nu = inv_nu;
    const RadialBf16 bfw = W.bf16_view();
    w.r_compact[t] = r_compact_for(M, chunks, keep_A) ? 1 : 0;
    const EdgePairs prs = graph_pairs(G, w.r_compact[t]);
    ta.r_row = w.r_compact[t] ? G->pair_of->as<int>() : nullptr;
    for (const RChunk& ch : chunks) {
      void* Rc = chunk_r(w, t, R, ch, PCu, lr_bf16 ? 2 : 4);
      {
        ProfScope ps(&M->prof, stage_id(kRadialFwd, t), st);
        launch_radial_fwd(c.n_basis, dvec, row_ptr, N, Ecap, W.rad1.as<float>(), W.rad2.as<float>(),
                          W.rad3.as<float>(), L.p_full * C, PCu, Rc, lr_bf16, rc, p_env, bf16, st, ch.e0, ch.e1,
                          &bfw, pairs_for(M, ch, prs));
      }
      set_chunk(ta, ch);
      ta.R = static_cast<const float*>(Rc);
      ProfScope ps(&M->prof, stage_id(kTpFwd, t), st);
      launch_tp(0, ta, st);
    }
    float* ht = w.ht[t]->as<float>();
    const int split = (!prod && L.nc_out == 1) ? mix_split_parts(L.p_used_l3[0] * C + (hin ? C : 0)) : 1;
    int n_parts = 0;
    {
      ProfScope ps(&M->prof, stage_id(kMixFwd, t), st);
      if (prod) {
        launch_mix(M, L, W, A, nullptr, w.at[t]->as<float>(), L.nc_a, N, st, bf16);
      } else if (split > 1) {
        float* part = ensure(w.mixp, &M->alloc, sizeof(float) * (size_t)split * N * C).as<float>();
        n_parts = launch_mix_scalar_split(M, L, W, A, hin, part, split, N, st, bf16);
      } else {
        launch_mix(M, L, W, A, hin, ht, L.nc_out, N, st, bf16);
      }
    }
    if (prod) product_tail(t, L, W, hin, ht);
    if (defer_last_gate && t == T && !prod && L.nc_out == 1) {
      w.last_parts = n_parts;
      continue;
    }
    {
      ProfScope ps(&M->prof, stage_id(kGateFwd, t), st);
      if (n_parts > 0)
        launch_gate_fwd_sum(w.mixp->as<float>(), n_parts, ht, w.h[t]->as<float>(), N, C, st);
      else
        launch_gate_fwd(ht, w.h[t]->as<float>(), N, L.nc_out, C, st);
    }
  }
}

void energy_forces(e3mi_model* M, e3mi_graph* G, const double* pos, double* energy, float* forces,
                   double* atom_energy, hipStream_t st) {
  const Config& c = M->cfg;
  const int N = G->N, S = G->S, C = c.channels, T = c.layers;
  const long Ecap = G->E_room;  // edge capacity (>= the skin-list count)
  const float inv_nu = (float)(1.0 / c.avg_neighbors);
  const float rc = (float)c.cutoff;
  const int p_env = c.envelope_p;
  Workspace& w = M->ws;
  if (N == 0) {
    launch_zero(energy, sizeof(double) * S, st);
    return;
  }
  const bool coulomb = c.coulomb;
  // the readout applies the last layer's gate and its adjoint itself, unless
  // the charge adjoint must still be added to dE/dh between the two
  const bool gate_in_readout = T >= 2 && !coulomb && c.correlation != 2 && M->plans[T - 1].nc_out == 1;
  w.last_parts = -1;
  forward_pass(M, G, pos, false, st, M->precision == E3MI_BF16_MIX, gate_in_readout);
  const int* row_ptr = G->row_ptr_x->as<int>();
  const int* src = G->src_x->as<int>();
  const float4* dvec = G->dvec_x->as<float4>();
  const int* species = G->species->as<int>();
  float* A = w.A->as<float>();
  float* dcur = w.dh_a->as<float>();
  float* dother = w.dh_b->as<float>();
  if (coulomb) {
    E3MI_REQUIRE(G->ctiles, E3MI_EINVAL, "graph was built for a model without the Coulomb term");
    for (auto* b : {&w.q_raw, &w.q, &w.pot}) ensure(*b, &M->alloc, sizeof(float) * (size_t)N);
    ensure(w.fc, &M->alloc, sizeof(float) * 3 * (size_t)N);
    ensure(w.pot_mean, &M->alloc, sizeof(float) * (size_t)S);
  }
  if (gate_in_readout) {
    E3MI_REQUIRE(w.last_parts >= 0, E3MI_EINVAL, "internal: last layer was not left before its gate");
    ProfScope ps(&M->prof, stage_id(kReadout), st);
    launch_readout_gated(w.last_parts > 0 ? w.mixp->as<float>() : w.ht[T]->as<float>(), w.last_parts, species,
                         M->read1->as<float>(), M->read2->as<float>(), M->e0->as<float>(), N, C,
                         w.e_atom->as<double>(), w.dht->as<float>(), st);
    launch_energy(w.e_atom->as<double>(), G->off_d->as<int64_t>(), S, energy, st);
  } else {
    ProfScope ps(&M->prof, stage_id(kReadout), st);
    launch_readout(w.h[T]->as<float>(), M->plans[T - 1].nc_out, species, M->read1->as<float>(),
                   M->read2->as<float>(), M->e0->as<float>(), N, C, w.e_atom->as<double>(), dcur, st,
                   coulomb ? M->qhead->as<float>() : nullptr, coulomb ? M->qbias->as<float>() : nullptr,
                   coulomb ? w.q_raw->as<float>() : nullptr);
    if (!coulomb) launch_energy(w.e_atom->as<double>(), G->off_d->as<int64_t>(), S, energy, st);
  }
  if (coulomb) {
    const int64_t* offd = G->off_d->as<int64_t>();
    launch_charge_fix(w.q_raw->as<float>(), offd, G->charge->as<double>(), S, w.q->as<float>(), st);
    {
      ProfScope ps(&M->prof, stage_id(kCoulomb), st);
      launch_coulomb(G->ctiles->as<int2>(), G->n_ctiles, G->c_waves, offd, pos, w.q->as<float>(), (float)c.soft_core_r0,
                     w.e_atom->as<double>(), w.pot->as<float>(), w.fc->as<float>(), st);
    }
    launch_coulomb_dq(offd, G->owner->as<int>(), S, N, w.pot->as<float>(), w.pot_mean->as<float>(),
                      M->qhead->as<float>(), C, dcur, st);
    launch_energy(w.e_atom->as<double>(), offd, S, energy, st);
  }
  if (atom_energy)
    E3MI_HIP(hipMemcpyAsync(atom_energy, w.e_atom->p, sizeof(double) * N, hipMemcpyDeviceToDevice, st));

  // ---- adjoint: dE/dr ----
  float* dht = w.dht->as<float>();
  float4* g = w.g->as<float4>();
  const bool fact = factorised_first(M);
  const int S64 = c.n_species * c.radial_hidden;
  const bool prod = c.correlation == 2;
  const bool bf16 = M->precision == E3MI_BF16_MIX;
  for (int t = T; t >= 1; --t) {
    const LayerPlan& L = M->plans[t - 1];
    LayerWeights& W = *M->lw[t - 1];
    const float* hin = w.h[t - 1]->as<float>();
    const int PCu = L.p_used * C;
    if (!(gate_in_readout && t == T)) {
      ProfScope ps(&M->prof, stage_id(kGateBwd, t), st);
      launch_gate_bwd(w.ht[t]->as<float>(), dcur, dht, N, L.nc_out, C, st);
    }
    // product block: dB = dh~ W_lin^T (the self-connection part goes to the
    // previous layer's gradient), then dA~; the mix adjoint starts from dA~
    const float* dmix = dht;
    int dmix_nc = L.nc_out;
    if (prod) {
      {
        ProfScope ps(&M->prof, stage_id(kMixBwd, t), st);
        if (t > 1) launch_zero(dother, sizeof(float) * (size_t)N * L.nc_in * C, st);
        launch_lin_adjoint(M, L, W, dht, w.Bp->as<float>(), t > 1 ? dother : nullptr, N, st, bf16);
      }
      ProductArgs pa = product_args(M, G, L, W, w.at[t]->as<float>());
      pa.dB = w.Bp->as<float>();
      pa.dat = w.dat->as<float>();
      {
        ProfScope ps(&M->prof, stage_id(kProductBwd, t), st);
        launch_product(false, pa, st);
      }
      dmix = w.dat->as<float>();
      dmix_nc = L.nc_a;
    }
    if (t == 1 && fact) {
      float* dG1 = w.dG1->as<float>();
      {
        ProfScope ps(&M->prof, stage_id(kMixBwd, 1), st);
        GemmArgs grp[kMaxGemmGroup];
        int n = 0;
        for (int l3 = 0; l3 <= L.l3max_used; ++l3) {
          const int gg = 2 * l3 + 1;
          GemmArgs& ga = grp[n++] = GemmArgs{};
          ga.a0 = RowMap{const_cast<float*>(dmix) + (long)l3 * l3 * C, (long)dmix_nc * C, (long)C, gg};
          ga.b0 = M->UT[l3]->as<float>();
          ga.ldb0 = S64;
          ga.k0 = C;
          ga.c = RowMap{dG1 + (long)l3 * l3 * S64, (long)L.nc_a * S64, (long)S64, gg};
          ga.M = N * gg;
          ga.Nc = S64;
        }
        launch_gemm_group(grp, n, st, M->precision == E3MI_BF16_MIX);
      }
      {
        ProfScope ps(&M->prof, stage_id(kFirstBwd, 1), st);
        launch_first(false, c.lmax, L.l3max_used, row_ptr, src, dvec, species, N, S64, W.rad1.as<float>(),
                     W.rad2T.as<float>(), first_pair_index(M, G), w.P2f->as<float>(), nullptr, dG1, g,
                     T != 1 ? 1 : 0, rc, p_env, st);
      }
      continue;
    }
    {
      ProfScope ps(&M->prof, stage_id(kMixBwd, t), st);
      // the per-edge node adjoint writes the components of dh the self
      // connection's adjoint leaves alone, so only the fused layer needs dh cleared
      if (t > 1 && !prod && fused_last(M, L, false, bf16))
        launch_zero(dother, sizeof(float) * (size_t)N * L.nc_in * C, st);
      launch_mix_adjoint(M, L, W, dmix, dmix_nc, A, (t > 1 && !prod) ? dother : nullptr, N, st, bf16);
    }
    if (fused_last(M, L, false, M->precision == E3MI_BF16_MIX)) {
      LastArgs la = last_args(M, G, L, W, hin);
      la.dA = A;
      la.g = g;
      la.accumulate = t != T ? 1 : 0;
      la.dh = dother;
      {
        ProfScope ps(&M->prof, stage_id(kLastBwd, t), st);
        launch_last(false, la, st);
      }
      std::swap(dcur, dother);
      continue;
    }
    const float* R = w.R[t]->as<float>();  // BF16 values when r_bf16
    const bool r_bf16 = r_bf16_layer(w, L);
    TpArgs ta{};
    const bool lr_bf16 = r_bf16_layer(w, L);
    ta.r_bf16 = lr_bf16 ? 1 : 0;
    ta.lmax = c.lmax;
    ta.kind = L.kind;
    ta.cpt = cpt_for(L, C);
    ta.row_ptr = row_ptr;
    ta.src = src;
    ta.dvec = dvec;
    ta.R = R;
    ta.r_stride = PCu;
    ta.h = hin;
    ta.h_nc = L.nc_in;
    ta.dA = A;
    ta.dR = w.dR->as<float>();
    ta.dY = w.dY->as<float>();
    ta.N = N;
    ta.C = C;
    ta.inv_nu = inv_nu;
    ta.dh = dother;
    ta.dh_nc = L.nc_in;
    if (!prod) {
      const int l_sc = std::min(L.l3max_used, L.l1max);  // orders the self-connection adjoint wrote
      ta.dh_acc = (l_sc + 1) * (l_sc + 1);
    }
    // layers with every path: the edge adjoint, which holds dA_i, also writes
    // each edge's sender-gradient message (16 x C values per edge), which a
    // node pass adds up per sender, instead of a node adjoint gathering the
    // receivers' dA rows (99 x C values per edge)
    const bool use_msg = L.kind == 1 && t > 1;  // kind 1: every path
    if (use_msg) {
      ta.msg = ensure(w.msg, &M->alloc, sizeof(float) * r_chunk_edges(M, Ecap, PCu) * L.nc_in * C).as<float>();
      ta.touched = ensure(w.touched, &M->alloc, sizeof(int) * ((size_t)N + 1)).as<int>();
    }
    // with more than one chunk R is recomputed chunk by chunk (the forward
    // pass kept only the last chunk), unless it was kept whole
    const std::vector<RChunk> chunks = r_chunks(M, G, PCu, st);
    const bool recompute = chunks.size() > 1 && !w.r_whole[t];
    const RadialBf16 bfw = W.bf16_view();
    const EdgePairs prs = graph_pairs(G);
    ta.rev = G->rev_x->as<int>();
    ta.r_row = w.r_compact[t] ? G->pair_of->as<int>() : nullptr;
    // scalar-output layer: the sender-side adjoint gives dR, dY and dh in one
    // pass (chunk by chunk: a chunk's receivers are the senders whose rows it holds)
    const bool sender_side = tps_supported(ta);
    for (const RChunk& ch : chunks) {
      ta.R = static_cast<const float*>(chunk_r(w, t, w.R[t]->p, ch, PCu, r_bf16 ? 2 : 4));
      if (sender_side) {
        if (recompute) {
          ProfScope ps(&M->prof, stage_id(kRadialFwd, t), st);
          launch_radial_fwd(c.n_basis, dvec, row_ptr, N, Ecap, W.rad1.as<float>(), W.rad2.as<float>(),
                            W.rad3.as<float>(), L.p_full * C, PCu, w.R[t]->p, r_bf16, rc, p_env, bf16, st, ch.e0,
                            ch.e1, &bfw);
        }
        set_chunk(ta, ch);
        TpArgs ts = ta;
        if (t == 1) ts.dh = nullptr;
        {
          ProfScope ps(&M->prof, stage_id(kTpBwdEdge, t), st);
          launch_tps_sender(ts, st);
        }
        ProfScope ps(&M->prof, stage_id(kRadialBwd, t), st);
        launch_radial_bwd(c.n_basis, c.lmax, dvec, row_ptr, N, Ecap, W.rad1.as<float>(), W.rad2.as<float>(),
                          W.rad2T.as<float>(), W.rad3T.as<float>(), PCu, w.dR->p, r_bf16, w.dY->as<float>(), g,
                          t != T ? 1 : 0, rc, p_env, bf16, st, ch.e0, ch.e1, &bfw, pairs_for(M, ch, prs));
        continue;
      }
      if (recompute) {
        ProfScope ps(&M->prof, stage_id(kRadialFwd, t), st);
        launch_radial_fwd(c.n_basis, dvec, row_ptr, N, Ecap, W.rad1.as<float>(), W.rad2.as<float>(),
                          W.rad3.as<float>(), L.p_full * C, PCu, w.R[t]->p, r_bf16, rc, p_env, bf16, st, ch.e0,
                          ch.e1, &bfw);
      }
      set_chunk(ta, ch);
      ta.tag = (int)(++w.msg_tag & 0x7fffffffu);
      {
        ProfScope ps(&M->prof, stage_id(kTpBwdEdge, t), st);
        launch_tp(1, ta, st);
      }
      {
        ProfScope ps(&M->prof, stage_id(kRadialBwd, t), st);
        launch_radial_bwd(c.n_basis, c.lmax, dvec, row_ptr, N, Ecap, W.rad1.as<float>(), W.rad2.as<float>(),
                          W.rad2T.as<float>(), W.rad3T.as<float>(), PCu, w.dR->p, r_bf16, w.dY->as<float>(), g,
                          t != T ? 1 : 0, rc, p_env, bf16, st, ch.e0, ch.e1, &bfw, pairs_for(M, ch, prs));
      }
      if (t > 1) {
        ProfScope ps(&M->prof, stage_id(kTpBwdNode, t), st);
        launch_tp(use_msg ? 7 : 2, ta, st);
      }
    }
    if (t > 1) std::swap(dcur, dother);
  }
  {
    ProfScope ps(&M->prof, stage_id(kForces), st);
    launch_forces(row_ptr, G->rev_x->as<int>(), g, N, forces, st, coulomb ? w.fc->as<float>() : nullptr);
  }
}

size_t footprint(const e3mi_model* M, int64_t n_atoms, int64_t n_edges) {
  const Config& c = M->cfg;
  // edge buffers: the skin edges, plus the 1/8 room a rebuild that outgrows them adds
  const size_t n_e = (size_t)std::max<int64_t>(n_edges, 0);
  const size_t N = (size_t)std::max<int64_t>(n_atoms, 0), E = n_e + n_e / 8 + 65;
  const size_t C = c.channels, NC = (size_t)(c.lmax + 1) * (c.lmax + 1);
  size_t b = 0;
  b += E * (8 + 4 * 3) + E * (4 + 16 + 4 + 4 + 4);   // skin list + pruned list
  b += N * (4 * 4 + 24 + 8) + 64 * 1024;             // per-atom graph data
  size_t a_max = 0, dr_max = 0, msg_max = 0, kept = 0;
  b += N * C * 4;                                    // embedding
  const bool bf16 = M->precision == E3MI_BF16_MIX;
  for (int t = 1; t <= c.layers; ++t) {
    const LayerPlan& L = M->plans[t - 1];
    b += 2 * N * L.nc_out * C * 4;
    if (L.n_prod) b += N * L.nc_a * C * 4;  // A~ kept for the product block's adjoint
    a_max = std::max(a_max, (size_t)L.a_per_atom);
    if (t == 1 && factorised_first(M)) {
      b += 2 * N * L.nc_out * (size_t)c.n_species * c.radial_hidden * 4;  // G and dG
      b += E * (size_t)c.radial_hidden * 4;                                // hidden pre-activations
      continue;
    }
    if (fused_last(M, L, false, bf16)) continue;  // no per-edge R
    // R (FP32 bound) of every edge, or of one receiver chunk unless kept whole
    // (n_edges stands for the edges inside the cutoff); dR and the
    // sender-gradient messages of a full layer per chunk
    const size_t PCu = (size_t)L.p_used * C;
    const size_t chunk = std::min(E, M->r_chunk_bytes / (PCu * 4));
    bool whole = chunk >= E;
    if (!whole && kept + E * PCu * 4 <= M->r_keep_bytes) {
      whole = true;
      kept += E * PCu * 4;
    }
    b += (whole ? E : chunk) * PCu * 4;
    dr_max = std::max(dr_max, chunk * PCu * 4);
    if (L.kind == 1 && t > 1) msg_max = std::max(msg_max, chunk * L.nc_in * C * 4);
  }
  b += N * a_max * 4 + dr_max + msg_max + E * (64 + 16) + 3 * N * NC * C * 4 + N * 8;
  if (c.correlation == 2) b += 2 * N * NC * C * 4;  // B / dB and dA~
  return b;
}

// Offsets of every weight tensor in the flat FP64 vector (file order).
struct WeightOffsets {
  size_t emb = 0, read1 = 0, read2 = 0, e0 = 0, qhead = 0, qbias = 0, total = 0;
  std::vector<size_t> sym1, sym2;
  std::vector<std::array<size_t, 4>> lin;
  std::vector<size_t> rad1, rad2, rad3;
  std::vector<std::array<size_t, 4>> mix, self_;
};

WeightOffsets weight_offsets(const Config& c) {
  WeightOffsets o;
  const size_t C = c.channels, H = c.radial_hidden;
  size_t cur = 0;
  o.emb = cur;
  cur += (size_t)c.n_species * C;
  for (int t = 1; t <= c.layers; ++t) {
    const LayerPlan L = plan_layer(c, t);
    o.rad1.push_back(cur);
    cur += (size_t)c.n_basis * H;
    o.rad2.push_back(cur);
    cur += H * H;
    o.rad3.push_back(cur);
    cur += H * (size_t)L.p_full * C;
    std::array<size_t, 4> m{}, sf{};
    for (int l3 = 0; l3 <= c.lmax; ++l3) {
      m[l3] = cur;
      cur += (size_t)L.p_full_l3[l3] * C * C;
    }
    for (int l = 0; l <= L.l1max; ++l) {
      sf[l] = cur;
      cur += C * C;
    }
    o.mix.push_back(m);
    o.self_.push_back(sf);
    std::array<size_t, 4> ln{};
    o.sym1.push_back(cur);
    o.sym2.push_back(cur);
    if (L.n_prod) {
      cur += (size_t)c.n_species * (L.lout + 1) * C;
      o.sym2.back() = cur;
      cur += (size_t)c.n_species * L.n_prod * C;
      for (int l = 0; l <= L.lout; ++l) {
        ln[l] = cur;
        cur += C * C;
      }
    }
    o.lin.push_back(ln);
  }
  o.read1 = cur;
  cur += C * c.readout_hidden;
  o.read2 = cur;
  cur += c.readout_hidden;
  o.e0 = cur;
  cur += c.n_species;
  if (c.coulomb) {
    o.qhead = cur;
    cur += C;
    o.qbias = cur;
    cur += c.n_species;
  }
  o.total = cur;
  return o;
}

// Convert the FP64 weights to FP32 device tensors (and the transposed copies
// the adjoint GEMMs read). Buffers are reused when they exist.
void upload_weights(e3mi_model* M, const double* wts) {
  const Config& c = M->cfg;
  Allocator* a = &M->alloc;
  const int C = c.channels, H = c.radial_hidden;
  size_t cur = 0;
  auto take = [&](size_t cnt) {
    std::vector<float> v(cnt);
    for (size_t i = 0; i < cnt; ++i) v[i] = (float)wts[cur + i];
    cur += cnt;
    return v;
  };
  M->emb = upload_f32(a, take((size_t)c.n_species * C));
  for (int t = 1; t <= c.layers; ++t) {
    const LayerPlan L = plan_layer(c, t);
    if ((int)M->lw.size() < t) {
      M->plans.push_back(L);
      auto Wn = std::make_unique<LayerWeights>();
      for (DevBuf* b : {&Wn->rad1, &Wn->rad2, &Wn->rad2T, &Wn->rad3, &Wn->rad3T, &Wn->rad3u, &Wn->rad2b, &Wn->rad2Tb,
                        &Wn->rad3Tb, &Wn->rad3ub, &Wn->sym1, &Wn->sym2})
        b->a = a;
      for (int l = 0; l < 4; ++l)
        Wn->mix[l].a = Wn->mixT[l].a = Wn->self_[l].a = Wn->selfT[l].a = Wn->lin[l].a = Wn->linT[l].a = a;
      M->lw.push_back(std::move(Wn));
    }
    LayerWeights* W = M->lw[t - 1].get();
    auto up = [&](DevBuf& b, const std::vector<float>& v) {
      b.ensure(v.size() * sizeof(float));
      E3MI_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(float), hipMemcpyHostToDevice));
    };
    auto up16 = [&](DevBuf& b, const std::vector<float>& v) {
      std::vector<uint16_t> h(v.size());
      for (size_t k = 0; k < v.size(); ++k) h[k] = bf16_rne(v[k]);
      b.ensure(h.size() * sizeof(uint16_t));
      E3MI_HIP(hipMemcpy(b.p, h.data(), h.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    };
    const auto r1 = take((size_t)c.n_basis * H);
    const auto r2 = take((size_t)H * H);
    const auto r3 = take((size_t)H * L.p_full * C);
    up(W->rad1, r1);
    up(W->rad2, r2);
    up(W->rad2T, transpose(r2, H, H));
    up(W->rad3, r3);
    // transpose of the used columns only: [p_used C, H]
    std::vector<float> r3t((size_t)L.p_used * C * H);
    for (int k = 0; k < H; ++k)
      for (int col = 0; col < L.p_used * C; ++col) r3t[(size_t)col * H + k] = r3[(size_t)k * L.p_full * C + col];
    up(W->rad3T, r3t);
    // the used columns alone, row-major [H, p_used C]
    std::vector<float> r3u((size_t)H * L.p_used * C);
    for (int k = 0; k < H; ++k)
      for (int col = 0; col < L.p_used * C; ++col)
        r3u[(size_t)k * L.p_used * C + col] = r3[(size_t)k * L.p_full * C + col];
    up(W->rad3u, r3u);
    // BF16 copies (round to nearest even, as the device's conversion does)
    up16(W->rad2b, r2);
    up16(W->rad2Tb, transpose(r2, H, H));
    up16(W->rad3Tb, r3t);
    {
      // W3 (used columns) in slabs of 32 columns: [PC / 32][64][32]
      const int PCu = L.p_used * C;
      std::vector<float> r3s((size_t)H * PCu);
      for (int q = 0; q < H; ++q)
        for (int col = 0; col < PCu; ++col)
          r3s[((size_t)(col / 32) * H + q) * 32 + col % 32] = r3u[(size_t)q * PCu + col];
      up16(W->rad3ub, r3s);
    }
    for (int l3 = 0; l3 <= c.lmax; ++l3) {
      const int P3 = L.p_full_l3[l3];
      const auto m = take((size_t)P3 * C * C);
      if (l3 <= L.l3max_used) {
        up(W->mix[l3], m);
        up(W->mixT[l3], transpose(m, P3 * C, C));
      }
    }
    for (int l = 0; l <= L.l1max; ++l) {
      const auto s = take((size_t)C * C);
      up(W->self_[l], s);
      up(W->selfT[l], transpose(s, C, C));
    }
    if (L.n_prod) {
      up(W->sym1, take((size_t)c.n_species * (L.lout + 1) * C));
      up(W->sym2, take((size_t)c.n_species * L.n_prod * C));
      for (int l = 0; l <= L.lout; ++l) {
        const auto m = take((size_t)C * C);
        up(W->lin[l], m);
        up(W->linT[l], transpose(m, C, C));
      }
    }
  }
  M->read1 = upload_f32(a, take((size_t)C * c.readout_hidden));
  M->read2 = upload_f32(a, take((size_t)c.readout_hidden));
  M->e0 = upload_f32(a, take((size_t)c.n_species));
  if (c.coulomb) {
    M->qhead = upload_f32(a, take((size_t)C));
    M->qbias = upload_f32(a, take((size_t)c.n_species));
  }
  E3MI_REQUIRE(cur == weight_count(c), E3MI_EINVAL, "internal: weight cursor mismatch");
  // U_l = nu^-1 (W3[:, l C + k] W_emb[s, k]) W_mix_l, rows (s, q), in FP64.
  const WeightOffsets off = weight_offsets(c);
  const LayerPlan L1p = plan_layer(c, 1);
  const int S64 = c.n_species * H;
  for (int l = 0; l <= L1p.l3max_used; ++l) {
    std::vector<double> U((size_t)S64 * C, 0.0);
    const double* W3 = wts + off.rad3[0];
    const double* Wm = wts + off.mix[0][l];   // [C, C]: one path (0,l,l) per order
    const double* We = wts + off.emb;
    std::vector<double> V(C);
    for (int sp = 0; sp < c.n_species; ++sp)
      for (int q = 0; q < H; ++q) {
        for (int k = 0; k < C; ++k) V[k] = W3[(size_t)q * L1p.p_full * C + (size_t)l * C + k] * We[(size_t)sp * C + k];
        double* Ur = &U[((size_t)sp * H + q) * C];
        for (int k = 0; k < C; ++k) {
          const double v = V[k] / c.avg_neighbors;
          for (int kp = 0; kp < C; ++kp) Ur[kp] += v * Wm[(size_t)k * C + kp];
        }
      }
    std::vector<float> Uf(U.begin(), U.end());
    M->U[l] = upload_f32(a, Uf);
    M->UT[l] = upload_f32(a, transpose(Uf, S64, C));
  }
}

e3mi_model* new_model(const char* json, const double* wts, size_t n, int precision, e3mi_alloc_fn al,
                      e3mi_free_fn fr, void* ctx) {
  auto M = std::make_unique<e3mi_model>();
  M->cfg = parse_config(json);
  const Config& c = M->cfg;
  E3MI_REQUIRE(precision == E3MI_FP32 || precision == E3MI_BF16_MIX, E3MI_EINVAL, "unknown precision");
  M->precision = precision;
  E3MI_REQUIRE(wts, E3MI_EINVAL, "weights are NULL");
  const size_t expect = weight_count(c);
  E3MI_REQUIRE(n == expect, E3MI_EINVAL,
               "weight count " + std::to_string(n) + " does not match the configuration (" + std::to_string(expect) + ")");
  for (size_t i = 0; i < n; ++i) E3MI_REQUIRE(std::isfinite(wts[i]), E3MI_ENAN, "weights are not finite");
  M->alloc.alloc = al;
  M->alloc.free_fn = fr;
  M->alloc.ctx = ctx;
  upload_weights(M.get(), wts);
  return M.release();
}


// Second-order pass for s = sum_s gE_s E_s - D_v E (v = gF): forward (primal
// + tangent along v), then the reverse pass over both. out (may be NULL): the
// gradient of s with respect to every weight, i.e. the vector-Jacobian
// product of (E, F) -> weights for upstream (gE, gF). hv (may be NULL):
// -ds/dr, which for gE = 0 is the Hessian-vector product H v (the reverse pass
// is continued through each layer's edge geometry).
void second_order(e3mi_model* M, e3mi_graph* G, const double* pos, const double* gE, const float* gF, double* out,
                  float* hv, hipStream_t st, bool primal_ready = false) {
  const Config& c = M->cfg;
  Allocator* a = &M->alloc;
  const int N = G->N, C = c.channels, T = c.layers, H = c.radial_hidden;
  const long Ecap = G->E_room;  // edge capacity (>= the skin-list count)
  const int NC = (c.lmax + 1) * (c.lmax + 1);
  const float inv_nu = (float)(1.0 / c.avg_neighbors);
  const float rc = (float)c.cutoff;
  const int p_env = c.envelope_p;
  Workspace& w = M->ws;
  E3MI_REQUIRE(!c.coulomb, E3MI_EUNSUPPORTED,
               "second-order passes (parameter gradients, Hessian-vector products) of the Coulomb term are not implemented");
  const bool prod = c.correlation == 2;
  const WeightOffsets off = weight_offsets(c);
  if (out) E3MI_HIP(hipMemsetAsync(out, 0, sizeof(double) * off.total, st));
  if (N == 0) return;
  // primal_ready: the previous call on this graph and positions left the
  // primal values (h, h~, R, A per layer) in the workspace
  if (!primal_ready) forward_pass(M, G, pos, true, st, false);
  const int* row_ptr = G->row_ptr_x->as<int>();
  const int* src = G->src_x->as<int>();
  const float4* dvec = G->dvec_x->as<float4>();
  const int* rows_dev = row_ptr + N;  // number of edges inside the cutoff
  const size_t E1 = (size_t)Ecap + 1;

  // ---- workspace ----
  for (auto* v : {&w.Ad, &w.hd, &w.htd, &w.Rd, &w.P1d, &w.H1d, &w.P2d, &w.H2d}) v->resize(T + 1);
  long a_max = 0, pc_max = 0;
  for (int t = 1; t <= T; ++t) {
    const LayerPlan& L = M->plans[t - 1];
    ensure(w.Ad[t], a, sizeof(float) * (size_t)N * L.a_per_atom);
    ensure(w.hd[t], a, sizeof(float) * (size_t)N * L.nc_out * C);
    ensure(w.htd[t], a, sizeof(float) * (size_t)N * L.nc_out * C);
    ensure(w.Rd[t], a, sizeof(float) * E1 * L.p_used * C);
    for (auto* v : {&w.P1d, &w.H1d, &w.P2d, &w.H2d}) ensure((*v)[t], a, sizeof(float) * E1 * 2 * H);
    a_max = std::max(a_max, L.a_per_atom);
    pc_max = std::max(pc_max, (long)L.p_used * C);
  }
  ensure(w.dd, a, sizeof(float4) * E1);
  ensure(w.Bd, a, sizeof(float) * E1 * 16);
  for (auto* v : {&w.Prb, &w.Prc, &w.w2c}) ensure(*v, a, sizeof(float) * (size_t)N * 16);
  ensure(w.eb, a, sizeof(float) * (size_t)N);
  for (auto* v : {&w.xb, &w.xc, &w.hb_a, &w.hb_b, &w.hc_a, &w.hc_b}) ensure(*v, a, sizeof(float) * (size_t)N * NC * C);
  for (auto* v : {&w.Ab, &w.Ac}) ensure(*v, a, sizeof(float) * (size_t)N * a_max);
  for (auto* v : {&w.Rb, &w.Rc}) ensure(*v, a, sizeof(float) * E1 * pc_max);
  for (auto* v : {&w.P1g, &w.P2g}) ensure(*v, a, sizeof(float) * E1 * 2 * H);
  ensure(w.partial, a, sizeof(float) * std::max<size_t>(16u << 20, (size_t)H * pc_max));
  float* partial = w.partial->as<float>();
  if (hv) {
    for (auto* v : {&w.Ygb, &w.Ygc}) ensure(*v, a, sizeof(float) * E1 * 16);
    ensure(w.ghv, a, sizeof(float4) * E1);
  }
  if (prod) {
    w.atd.resize(T + 1);
    w.Bpd.resize(T + 1);
    long dw_max = 0;
    for (int t = 1; t <= T; ++t) {
      const LayerPlan& L = M->plans[t - 1];
      ensure(w.atd[t], a, sizeof(float) * (size_t)N * L.nc_a * C);
      ensure(w.Bpd[t], a, sizeof(float) * (size_t)N * (L.lout + 1) * (L.lout + 1) * C);
      dw_max = std::max(dw_max, (long)(L.lout + 1 + L.n_prod) * C);
    }
    for (auto* v : {&w.Bpb, &w.Bpc, &w.atb, &w.atc}) ensure(*v, a, sizeof(float) * (size_t)N * NC * C);
    if (out) ensure(w.dwp, a, sizeof(float) * (size_t)N * dw_max);
  }

  // ---- tangent forward along v = gF ----
  launch_edge_tangent(row_ptr, src, dvec, gF, N, w.dd->as<float4>(), st);
  const float4* dd = w.dd->as<float4>();
  for (int t = 1; t <= T; ++t) {
    const LayerPlan& L = M->plans[t - 1];
    LayerWeights& W = *M->lw[t - 1];
    const int PCu = L.p_used * C;
    launch_radial_dual_fwd(c.n_basis, dvec, dd, row_ptr, N, Ecap, W.rad1.as<float>(), W.rad2.as<float>(),
                           W.rad3.as<float>(), L.p_full * C, PCu, w.Rd[t]->as<float>(), w.Bd->as<float>(),
                           w.P1d[t]->as<float>(), w.H1d[t]->as<float>(), w.P2d[t]->as<float>(), w.H2d[t]->as<float>(),
                           rc, p_env, st);
    TpArgs ta{};
    ta.lmax = c.lmax;
    ta.kind = L.kind;
    ta.cpt = cpt_for(L, C);
    ta.row_ptr = row_ptr;
    ta.src = src;
    ta.dvec = dvec;
    ta.dd = dd;
    ta.R = w.R[t]->as<float>();
    ta.Rd = w.Rd[t]->as<float>();
    ta.r_stride = PCu;
    ta.h = w.h[t - 1]->as<float>();
    ta.hd = t > 1 ? w.hd[t - 1]->as<float>() : nullptr;
    ta.h_nc = L.nc_in;
    ta.Ad = w.Ad[t]->as<float>();
    ta.N = N;
    ta.C = C;
    ta.inv_nu = inv_nu;
    launch_tp(3, ta, st);
    if (prod) {
      // A~_dot = A_dot W_mix (no self connection), B_dot, then h~_dot = B_dot W_lin + h_dot S
      launch_mix(M, L, W, w.Ad[t]->as<float>(), nullptr, w.atd[t]->as<float>(), L.nc_a, N, st);
      ProductArgs pa = product_args(M, G, L, W, w.at[t]->as<float>());
      pa.atd = w.atd[t]->as<float>();
      pa.Bd = w.Bpd[t]->as<float>();
      launch_product_jvp(pa, st);
      launch_lin(M, L, W, w.Bpd[t]->as<float>(), t > 1 ? w.hd[t - 1]->as<float>() : nullptr, w.htd[t]->as<float>(),
                 N, st, false);
    } else {
      launch_mix(M, L, W, w.Ad[t]->as<float>(), t > 1 ? w.hd[t - 1]->as<float>() : nullptr,
                 w.htd[t]->as<float>(), L.nc_out, N, st);
    }
    launch_gate_dual_fwd(w.ht[t]->as<float>(), w.htd[t]->as<float>(), w.hd[t]->as<float>(), N, L.nc_out, C, st);
  }

  // ---- reverse: readout ----
  const int ncT = M->plans[T - 1].nc_out;
  float* hb = w.hb_a->as<float>();
  float* hc = w.hc_a->as<float>();
  float* hb2 = w.hb_b->as<float>();
  float* hc2 = w.hc_b->as<float>();
  launch_readout_dual(w.h[T]->as<float>(), w.hd[T]->as<float>(), ncT, G->owner->as<int>(), gE, M->read1->as<float>(),
                      M->read2->as<float>(), N, C, w.Prb->as<float>(), w.Prc->as<float>(), w.w2c->as<float>(), hb, hc,
                      w.eb->as<float>(), st);
  if (out) {
    launch_gemm_tn(RowMap{w.h[T]->as<float>(), (long)ncT * C, 0, 1}, RowMap{w.Prb->as<float>(), 16, 0, 1},
                   RowMap{w.hd[T]->as<float>(), (long)ncT * C, 0, 1}, RowMap{w.Prc->as<float>(), 16, 0, 1}, N,
                   nullptr, C, 16, partial, out + off.read1, 16, st);
    launch_group_sum(w.w2c->as<float>(), 16, nullptr, 1, N, 16, out + off.read2, 16, st);
    launch_group_sum(w.eb->as<float>(), 1, G->species->as<int>(), c.n_species, N, 1, out + off.e0, 1, st);
  }

  // ---- reverse: layers ----
  float* xb = w.xb->as<float>();
  float* xc = w.xc->as<float>();
  for (int t = T; t >= 1; --t) {
    const LayerPlan& L = M->plans[t - 1];
    LayerWeights& W = *M->lw[t - 1];
    const int PCu = L.p_used * C;
    const float* hin = w.h[t - 1]->as<float>();
    const float* hdin = t > 1 ? w.hd[t - 1]->as<float>() : nullptr;
    launch_gate_dual_bwd(w.ht[t]->as<float>(), w.htd[t]->as<float>(), hb, hc, xb, xc, N, L.nc_out, C, st);
    // weight gradients of the self connection (orders present in both h^{t-1} and h~)
    for (int l = 0; l <= (out ? std::min(L.l1max, prod ? L.lout : L.l3max_used) : -1); ++l) {
      const int g = 2 * l + 1;
      launch_gemm_tn(RowMap{const_cast<float*>(hin) + (long)l * l * C, (long)L.nc_in * C, (long)C, g},
                     RowMap{xb + (long)l * l * C, (long)L.nc_out * C, (long)C, g},
                     hdin ? RowMap{const_cast<float*>(hdin) + (long)l * l * C, (long)L.nc_in * C, (long)C, g}
                          : RowMap{nullptr, 0, 0, 1},
                     RowMap{xc + (long)l * l * C, (long)L.nc_out * C, (long)C, g}, (long)N * g, nullptr, C, C,
                     partial, out + off.self_[t - 1][l], C, st);
    }
    E3MI_HIP(hipMemsetAsync(hb2, 0, sizeof(float) * (size_t)N * L.nc_in * C, st));
    if (t > 1) E3MI_HIP(hipMemsetAsync(hc2, 0, sizeof(float) * (size_t)N * L.nc_in * C, st));
    // the mix's output adjoints (of A~ or h~, and of their tangents)
    const float* mb = xb;
    const float* mc = xc;
    int m_nc = L.nc_out;
    if (prod) {
      // h~ = B W_lin + h^{t-1} S: adjoints of B and B_dot (and of h^{t-1},
      // h_dot^{t-1} through S), W_lin's gradient from B and B_dot
      float* Bt = w.Bp->as<float>();
      ProductArgs pa = product_args(M, G, L, W, w.at[t]->as<float>());
      pa.atd = w.atd[t]->as<float>();
      if (out) {
        pa.B = Bt;
        launch_product(true, pa, st);  // B again (the forward pass keeps one layer's)
        for (int l = 0; l <= L.lout; ++l) {
          const int g = 2 * l + 1, nb = (L.lout + 1) * (L.lout + 1);
          launch_gemm_tn(RowMap{Bt + (long)l * l * C, (long)nb * C, (long)C, g},
                         RowMap{xb + (long)l * l * C, (long)L.nc_out * C, (long)C, g},
                         RowMap{w.Bpd[t]->as<float>() + (long)l * l * C, (long)nb * C, (long)C, g},
                         RowMap{xc + (long)l * l * C, (long)L.nc_out * C, (long)C, g}, (long)N * g, nullptr, C, C,
                         partial, out + off.lin[t - 1][l], C, st);
        }
      }
      launch_lin_adjoint(M, L, W, xb, w.Bpb->as<float>(), hb2, N, st, false);
      launch_lin_adjoint(M, L, W, xc, w.Bpc->as<float>(), t > 1 ? hc2 : nullptr, N, st, false);
      pa.Bb = w.Bpb->as<float>();
      pa.Bc = w.Bpc->as<float>();
      pa.atb = w.atb->as<float>();
      pa.atc = w.atc->as<float>();
      pa.dw = out ? w.dwp->as<float>() : nullptr;
      launch_product_dual_bwd(pa, st);
      if (out) {
        const long ldw = (long)(L.lout + 1 + L.n_prod) * C;
        launch_group_sum(pa.dw, ldw, G->species->as<int>(), c.n_species, N, (L.lout + 1) * C, out + off.sym1[t - 1],
                         (long)(L.lout + 1) * C, st);
        launch_group_sum(pa.dw + (long)(L.lout + 1) * C, ldw, G->species->as<int>(), c.n_species, N, L.n_prod * C,
                         out + off.sym2[t - 1], (long)L.n_prod * C, st);
      }
      mb = w.atb->as<float>();
      mc = w.atc->as<float>();
      m_nc = L.nc_a;
    }
    // weight gradients of the channel mix
    long gbase = 0;
    for (int l3 = 0; l3 <= (out ? L.l3max_used : -1); ++l3) {
      const int P3 = L.p_used_l3[l3], g = 2 * l3 + 1;
      launch_gemm_tn(RowMap{w.Al[t]->as<float>() + gbase, (long)g * P3 * C, (long)P3 * C, g},
                     RowMap{const_cast<float*>(mb) + (long)l3 * l3 * C, (long)m_nc * C, (long)C, g},
                     RowMap{w.Ad[t]->as<float>() + gbase, (long)g * P3 * C, (long)P3 * C, g},
                     RowMap{const_cast<float*>(mc) + (long)l3 * l3 * C, (long)m_nc * C, (long)C, g}, (long)N * g,
                     nullptr, P3 * C, C, partial, out + off.mix[t - 1][l3], C, st);
      gbase += (long)N * g * P3 * C;
    }
    // adjoints of A and A_dot; of h^{t-1} and h_dot^{t-1} through the self
    // connection (without the product block, the mix holds it)
    launch_mix_adjoint(M, L, W, mb, m_nc, w.Ab->as<float>(), prod ? nullptr : hb2, N, st);
    launch_mix_adjoint(M, L, W, mc, m_nc, w.Ac->as<float>(), (!prod && t > 1) ? hc2 : nullptr, N, st);
    // tensor product: adjoints of R and R_dot, then of h and h_dot
    TpArgs ta{};
    ta.lmax = c.lmax;
    ta.kind = L.kind;
    ta.cpt = cpt_for(L, C);
    ta.row_ptr = row_ptr;
    ta.src = src;
    ta.dvec = dvec;
    ta.dd = dd;
    ta.R = w.R[t]->as<float>();
    ta.Rd = w.Rd[t]->as<float>();
    ta.r_stride = PCu;
    ta.h = hin;
    ta.hd = hdin;
    ta.h_nc = L.nc_in;
    ta.Ab = w.Ab->as<float>();
    ta.Ac = w.Ac->as<float>();
    ta.Rb = w.Rb->as<float>();
    ta.Rc = w.Rc->as<float>();
    ta.hb = hb2;
    ta.hc = t > 1 ? hc2 : nullptr;
    ta.dh_nc = L.nc_in;
    ta.N = N;
    ta.C = C;
    ta.inv_nu = inv_nu;
    launch_tp(4, ta, st);
    launch_tp(5, ta, st);
    // radial MLP: adjoints of the pre-activations, then the weight gradients
    launch_radial_dual_bwd(row_ptr, N, Ecap, W.rad2T.as<float>(), W.rad3T.as<float>(), PCu, w.Rb->as<float>(),
                           w.Rc->as<float>(), w.P1d[t]->as<float>(), w.P2d[t]->as<float>(), w.P1g->as<float>(),
                           w.P2g->as<float>(), st);
    if (hv) {
      // continue to the positions through the harmonics and the radial basis
      ta.Yb = w.Ygb->as<float>();
      ta.Yc = w.Ygc->as<float>();
      launch_tp(6, ta, st);
      launch_hvp_geo(c.lmax, row_ptr, N, Ecap, dvec, dd, w.Ygb->as<float>(), w.Ygc->as<float>(), w.P1g->as<float>(),
                     W.rad1.as<float>(), rc, p_env, t != T ? 1 : 0, w.ghv->as<float4>(), st);
    }
    if (!out) {
      std::swap(hb, hb2);
      std::swap(hc, hc2);
      continue;
    }
    float* H2d = w.H2d[t]->as<float>();
    float* H1d = w.H1d[t]->as<float>();
    float* Bd = w.Bd->as<float>();
    float* P1g = w.P1g->as<float>();
    float* P2g = w.P2g->as<float>();
    launch_gemm_tn(RowMap{H2d, 2L * H, 0, 1}, RowMap{w.Rb->as<float>(), PCu, 0, 1}, RowMap{H2d + H, 2L * H, 0, 1},
                   RowMap{w.Rc->as<float>(), PCu, 0, 1}, Ecap, rows_dev, H, PCu, partial, out + off.rad3[t - 1],
                   (long)L.p_full * C, st);
    launch_gemm_tn(RowMap{H1d, 2L * H, 0, 1}, RowMap{P2g, 2L * H, 0, 1}, RowMap{H1d + H, 2L * H, 0, 1},
                   RowMap{P2g + H, 2L * H, 0, 1}, Ecap, rows_dev, H, H, partial, out + off.rad2[t - 1], H, st);
    launch_gemm_tn(RowMap{Bd, 16, 0, 1}, RowMap{P1g, 2L * H, 0, 1}, RowMap{Bd + 8, 16, 0, 1},
                   RowMap{P1g + H, 2L * H, 0, 1}, Ecap, rows_dev, c.n_basis, H, partial, out + off.rad1[t - 1], H,
                   st);
    std::swap(hb, hb2);
    std::swap(hc, hc2);
  }
  // embedding: h^0_i = W_emb[z_i]
  if (out) launch_group_sum(hb, C, G->species->as<int>(), c.n_species, N, C, out + off.emb, C, st);
  if (hv) launch_forces(row_ptr, G->rev_x->as<int>(), w.ghv->as<float4>(), N, hv, st);
}

void param_grad(e3mi_model* M, e3mi_graph* G, const double* pos, const double* gE, const float* gF, double* out,
                hipStream_t st) {
  E3MI_REQUIRE(out, E3MI_EINVAL, "null output");
  second_order(M, G, pos, gE, gF, out, nullptr, st);
}

// H v_k = d(grad E . v_k)/dr for k < n_vec (v, hv: [n_vec, N, 3]): the
// second-order pass with no energy seed, continued to the positions; the
// primal forward pass runs once for all directions.
void hessian_vectors(e3mi_model* M, e3mi_graph* G, const double* pos, int n_vec, const float* v, float* hv,
                     hipStream_t st) {
  E3MI_REQUIRE(v && hv, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(n_vec >= 0, E3MI_EINVAL, "n_vec must be >= 0");
  Workspace& w = M->ws;
  ensure(w.zeroE, &M->alloc, sizeof(double) * (size_t)std::max(G->S, 1));
  E3MI_HIP(hipMemsetAsync(w.zeroE->p, 0, sizeof(double) * (size_t)std::max(G->S, 1), st));
  const size_t stride = 3 * (size_t)G->N;
  for (int k = 0; k < n_vec; ++k)
    second_order(M, G, pos, w.zeroE->as<double>(), v + k * stride, nullptr, hv + k * stride, st, k > 0);
}

// Replace the weights of a model (same configuration), e.g. after an optimiser step.
void set_weights(e3mi_model* M, const double* wts, size_t n) {
  const Config& c = M->cfg;
  E3MI_REQUIRE(wts, E3MI_EINVAL, "weights are NULL");
  E3MI_REQUIRE(n == weight_count(c), E3MI_EINVAL, "weight count does not match the configuration");
  for (size_t i = 0; i < n; ++i) E3MI_REQUIRE(std::isfinite(wts[i]), E3MI_ENAN, "weights are not finite");
  E3MI_HIP(hipDeviceSynchronize());  // no kernel may still read the old weights
  upload_weights(M, wts);
}

// ---- MD -----------------------------------------------------------------------------------

constexpr double kAccelUnit = 0.009648533;  // angstrom/fs^2 per (eV/angstrom)/amu
constexpr double kBoltzmannEv = 8.617333262e-5;  // eV/K
constexpr double kBarEvA3 = 6.241509074e-7;        // eV/A^3 per bar

// Philox4x64-10 (Salmon et al., SC'11) on the host, for the barostat's two
// uniforms per volume proposal: key (seed, 1), counter (move, 0, 0, 0).
void philox4x64_10_host(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    const unsigned __int128 p0 = (unsigned __int128)M0 * c[0], p1 = (unsigned __int128)M1 * c[2];
    const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c[1] ^ k0, n2 = (uint64_t)(p0 >> 64) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint64_t)p1;
    c[2] = n2;
    c[3] = (uint64_t)p0;
    k0 += W0;
    k1 += W1;
  }
}

// Positions are never wrapped: the cell list bins wrapped copies internally and
// the image vectors refer to the raw positions, so a trajectory does not
// depend on when its rebuilds happen (a request gives the same bits alone and
// packed with others).
void md_rebuild(e3mi_md* D, hipStream_t st) {
  e3mi_graph* G = D->graph;
  ProfScope ps(&D->model->prof, stage_id(kGraphBuild), st);
  build_lists(G, D->x->as<double>(), st);
  D->since_build = 0;
  D->rebuild_next = false;
  D->rebuilds++;
}

e3mi_md* new_md(e3mi_model* M, int S, const int64_t* off, const double* pos, const double* vel,
                const int32_t* species, const double* masses, const double* cell, const uint8_t* pbc, double cutoff,
                double skin, int rebuild_every, hipStream_t st) {
  E3MI_REQUIRE(M && masses, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(rebuild_every >= 1, E3MI_EINVAL, "rebuild_every must be >= 1");
  for (int z = 0; z < M->cfg.n_species; ++z)
    E3MI_REQUIRE(masses[z] > 0 && std::isfinite(masses[z]), E3MI_EINVAL, "masses must be positive");
  auto D = std::make_unique<e3mi_md>();
  D->model = M;
  D->S = S;
  D->rebuild_every = rebuild_every;
  D->cutoff = cutoff;
  D->skin = skin;
  Allocator* a = &M->alloc;
  E3MI_REQUIRE(off && S >= 1, E3MI_EINVAL, "bad atom_offsets");
  E3MI_REQUIRE(cell && pbc, E3MI_EINVAL, "null cell or pbc");
  D->N = (int)off[S];
  E3MI_REQUIRE(D->N == 0 || (pos && vel && species), E3MI_EINVAL, "null state arrays");
  const size_t n3 = sizeof(double) * 3 * (D->N + 1);
  D->x = std::make_unique<DevBuf>(a);
  D->x->ensure(n3);
  D->v = std::make_unique<DevBuf>(a);
  D->v->ensure(n3);
  D->F = std::make_unique<DevBuf>(a);
  D->F->ensure(sizeof(float) * 3 * (D->N + 1));
  D->species = std::make_unique<DevBuf>(a);
  D->species->ensure(sizeof(int) * (D->N + 1));
  if (D->N) {
    E3MI_HIP(hipMemcpyAsync(D->x->p, pos, sizeof(double) * 3 * D->N, hipMemcpyDeviceToDevice, st));
    E3MI_HIP(hipMemcpyAsync(D->v->p, vel, sizeof(double) * 3 * D->N, hipMemcpyDeviceToDevice, st));
    E3MI_HIP(hipMemcpyAsync(D->species->p, species, sizeof(int) * D->N, hipMemcpyDeviceToDevice, st));
  }
  std::vector<double> inv((size_t)M->cfg.n_species);
  for (int z = 0; z < M->cfg.n_species; ++z) inv[z] = 1.0 / masses[z];
  D->inv_mass = upload(a, inv.data(), sizeof(double) * inv.size());
  D->energy = std::make_unique<DevBuf>(a);
  D->energy->ensure(sizeof(double) * S);
  D->flag = std::make_unique<DevBuf>(a);
  D->flag->ensure(3 * sizeof(unsigned long long));
  E3MI_HIP(hipMemsetAsync(D->flag->p, 0, 3 * sizeof(unsigned long long), st));
  D->v_prev = std::make_unique<DevBuf>(a);
  D->v_prev->ensure(n3);
  E3MI_HIP(hipHostMalloc((void**)&D->flag_host, 3 * sizeof(unsigned long long), hipHostMallocDefault));
  for (int k = 0; k < 3; ++k) D->flag_host[k] = 0;
  E3MI_HIP(hipEventCreateWithFlags(&D->drift_ev, hipEventDisableTiming));
  D->off_h.assign(off, off + S + 1);
  D->cell_h.assign(cell, cell + 9 * (size_t)S);
  D->pbc_h.assign(pbc, pbc + 3 * (size_t)S);
  D->graph = new_graph(M, S, off, D->x->as<double>(), D->species->as<int>(), cell, pbc, cutoff, skin, st);
  energy_forces(M, D->graph, D->x->as<double>(), D->energy->as<double>(), D->F->as<float>(), nullptr, st);
  E3MI_HIP(hipStreamSynchronize(st));
  return D.release();
}

void barostat_move(e3mi_md* D, const std::vector<int>& active, hipStream_t st);

void md_step(e3mi_md* D, int n_steps, double dt, double* energy_out, hipStream_t st) {
  E3MI_REQUIRE(n_steps >= 0 && std::isfinite(dt), E3MI_EINVAL, "bad step arguments");
  e3mi_graph* G = D->graph;
  const double hk = 0.5 * dt * kAccelUnit;
  const double lim = 0.5 * D->skin;
  const bool langevin = D->gamma > 0;
  const double c1 = std::exp(-D->gamma * dt), c2 = std::sqrt(std::max(0.0, 1.0 - c1 * c1));
  unsigned long long* flag = reinterpret_cast<unsigned long long*>(D->flag->p);
  for (int s = 0; s < n_steps; ++s) {
    const unsigned long long stamp = ++D->stamp;
    unsigned long long* probe = flag + 1 + (stamp & 1);
    unsigned long long* probe_next = flag + 1 + ((stamp + 1) & 1);
    {
      ProfScope ps(&D->model->prof, stage_id(kMdUpdate), st);
      if (!langevin) {
        launch_kick_drift(D->v->as<double>(), D->F->as<float>(), D->species->as<int>(), D->inv_mass->as<double>(),
                          hk, D->x->as<double>(), G->x_ref->as<double>(), dt, lim * lim, D->N, flag, stamp, probe, dt,
                          st);
      } else {
        // BAOAB: half kick and half drift, Ornstein-Uhlenbeck velocity update, half drift
        launch_kick_drift(D->v->as<double>(), D->F->as<float>(), D->species->as<int>(), D->inv_mass->as<double>(),
                          hk, D->x->as<double>(), G->x_ref->as<double>(), 0.5 * dt,
                          std::numeric_limits<double>::infinity(), D->N, flag, stamp, nullptr, 0.0, st);
        launch_ou(D->v->as<double>(), D->species->as<int>(), D->inv_mass->as<double>(), G->owner->as<int>(),
                  G->off_d->as<int64_t>(), D->seeds->as<uint64_t>(), D->step0->as<int64_t>(), D->steps, c1, c2,
                  kBoltzmannEv * D->temperature * kAccelUnit, D->N, st);
        launch_drift(D->x->as<double>(), D->v->as<double>(), G->x_ref->as<double>(), 0.5 * dt, lim * lim, D->N, flag,
                     stamp, probe, dt, st);
      }
    }
    // Rebuild every rebuild_every steps, and early on any step whose drift
    // takes an atom more than skin/2 from where the lists were built (a pair
    // could then be inside the cutoff without being listed). The early check
    // is decided before the step's results count: the force evaluation is
    // queued at once, the host waits only for the drift (so the device keeps
    // the evaluation to work on), and if the drift overran, the velocities are
    // put back to before the kick and the evaluation and kick are redone on
    // new lists. A rebuild does not change the selected edges or their order,
    // so the redone step equals one whose lists were exact throughout. So that
    // redoing stays rare, the drift's forecast of the next step's largest
    // displacement brings the rebuild forward to the next step when it
    // reaches skin/2.
    const bool scheduled = ++D->since_build >= D->rebuild_every || D->rebuild_next;
    if (scheduled) {
      md_rebuild(D, st);
    } else {
      E3MI_HIP(hipMemcpyAsync(D->flag_host, flag, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
      E3MI_HIP(hipEventRecord(D->drift_ev, st));
    }
    // the last step of the call hands the energies out in its kick launch
    // (unless a barostat move may still change them)
    const bool copy_here = energy_out && s + 1 == n_steps && D->baro_interval <= 0;
    auto force_and_kick = [&]() {
      energy_forces(D->model, G, D->x->as<double>(), D->energy->as<double>(), D->F->as<float>(), nullptr, st);
      ProfScope ps(&D->model->prof, stage_id(kMdUpdate), st);
      launch_kick_copy(D->v->as<double>(), D->F->as<float>(), D->species->as<int>(), D->inv_mass->as<double>(), hk,
                       D->N, D->energy->as<double>(), energy_out, copy_here ? D->S : 0,
                       scheduled ? nullptr : D->v_prev->as<double>(), probe_next, st);
    };
    force_and_kick();
    if (!scheduled) {
      E3MI_HIP(hipEventSynchronize(D->drift_ev));
      const volatile unsigned long long* fh = D->flag_host;
      if (fh[0] == stamp) {
        D->skin_violations++;
        if (D->N)
          E3MI_HIP(hipMemcpyAsync(D->v->p, D->v_prev->p, sizeof(double) * 3 * D->N, hipMemcpyDeviceToDevice, st));
        md_rebuild(D, st);
        force_and_kick();
      } else {
        const unsigned long long bits = fh[1 + (stamp & 1)];
        double f;
        std::memcpy(&f, &bits, sizeof f);
        D->rebuild_next = f > lim;
      }
    }
    if (copy_here) energy_out = nullptr;
    D->steps++;
    if (D->baro_interval > 0) {
      // each structure proposes on its own schedule, so the moves do not
      // depend on what else is packed with it
      std::vector<int> active((size_t)D->S);
      bool any = false;
      for (int q = 0; q < D->S; ++q) {
        active[q] = (D->step0_h[q] + D->steps) % D->baro_interval == 0;
        any |= active[q] != 0;
      }
      if (any) barostat_move(D, active, st);
    }
  }
  if (energy_out)
    E3MI_HIP(hipMemcpyAsync(energy_out, D->energy->p, sizeof(double) * D->S, hipMemcpyDeviceToDevice, st));
}

// One isotropic volume proposal per active structure, all evaluated in one
// pass and each decided alone (Metropolis on dE + P dV - N kB T ln V'/V);
// inactive structures are left as they are.
void barostat_move(e3mi_md* D, const std::vector<int>& active, hipStream_t st) {
  e3mi_graph* G = D->graph;
  e3mi_model* M = D->model;
  Allocator* a = &M->alloc;
  const int S = D->S, N = D->N;
  ProfScope ps(&M->prof, stage_id(kBarostat), st);
  std::vector<double> E_old(S), E_t(S), lam(S, 1.0), dV(S, 0.0), u1(S, 0.0);
  std::vector<int> ok(S, 1), keep(S, 1);
  E3MI_HIP(hipMemcpyAsync(E_old.data(), D->energy->p, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  E3MI_HIP(hipStreamSynchronize(st));
  const std::vector<double> box_old = G->box_h;
  for (int s = 0; s < S; ++s) {
    if (!active[s]) continue;
    uint64_t c[4] = {(uint64_t)D->baro_move[s], 0ull, 0ull, 0ull};
    philox4x64_10_host(c, D->baro_seed[s], 1ull);
    const double ua = ((double)(c[0] >> 11) + 0.5) * 0x1.0p-53, ub = ((double)(c[1] >> 11) + 0.5) * 0x1.0p-53;
    const double V = box_old[3 * s] * box_old[3 * s + 1] * box_old[3 * s + 2];
    dV[s] = (2.0 * ua - 1.0) * D->dv_max[s];
    u1[s] = ub;
    if (V + dV[s] > 0.0) {
      lam[s] = std::cbrt((V + dV[s]) / V);
    } else {
      ok[s] = 0;
      dV[s] = 0.0;
    }
    for (int k = 0; k < 3; ++k) G->box_h[3 * s + k] = box_old[3 * s + k] * lam[s];
  }
  ensure(D->x_save, a, sizeof(double) * 3 * (size_t)(N + 1));
  if (N) E3MI_HIP(hipMemcpyAsync(D->x_save->p, D->x->p, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, st));
  ensure(D->lam, a, sizeof(double) * S);
  ensure(D->keep, a, sizeof(int) * S);
  E3MI_HIP(hipMemcpyAsync(D->lam->p, lam.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
  launch_scale_positions(D->x->as<double>(), G->owner->as<int>(), D->lam->as<double>(), N, st);
  E3MI_HIP(hipMemcpyAsync(G->box_d->p, G->box_h.data(), sizeof(double) * 3 * S, hipMemcpyHostToDevice, st));
  build_lists(G, D->x->as<double>(), st);
  energy_forces(M, G, D->x->as<double>(), D->energy->as<double>(), D->F->as<float>(), nullptr, st);
  E3MI_HIP(hipMemcpyAsync(E_t.data(), D->energy->p, sizeof(double) * S, hipMemcpyDeviceToHost, st));
  E3MI_HIP(hipStreamSynchronize(st));
  const double kT = kBoltzmannEv * D->temperature, P = D->pressure_bar * kBarEvA3;
  bool all = true;
  for (int s = 0; s < S; ++s) {
    if (!active[s]) continue;
    const double V = box_old[3 * s] * box_old[3 * s + 1] * box_old[3 * s + 2];
    const double n_s = (double)(D->off_h[s + 1] - D->off_h[s]);
    keep[s] = 0;
    if (ok[s]) {
      const double w = (E_t[s] - E_old[s]) + P * dV[s] - n_s * kT * std::log((V + dV[s]) / V);
      keep[s] = (w <= 0.0 || u1[s] < std::exp(-w / kT)) ? 1 : 0;
    }
    D->baro_move[s]++;
    D->baro_proposed++;
    D->baro_accepted += keep[s];
    if (!keep[s]) {
      all = false;
      for (int k = 0; k < 3; ++k) G->box_h[3 * s + k] = box_old[3 * s + k];
    }
    for (int k = 0; k < 3; ++k) D->cell_h[9 * s + 4 * k] = G->box_h[3 * s + k];
  }
  if (!all) {
    // put the rejected structures back and evaluate the final state
    E3MI_HIP(hipMemcpyAsync(D->keep->p, keep.data(), sizeof(int) * S, hipMemcpyHostToDevice, st));
    launch_restore_rows(D->x->as<double>(), D->x_save->as<double>(), G->owner->as<int>(), D->keep->as<int>(), N, st);
    E3MI_HIP(hipMemcpyAsync(G->box_d->p, G->box_h.data(), sizeof(double) * 3 * S, hipMemcpyHostToDevice, st));
    build_lists(G, D->x->as<double>(), st);
    energy_forces(M, G, D->x->as<double>(), D->energy->as<double>(), D->F->as<float>(), nullptr, st);
  }
  E3MI_HIP(hipStreamSynchronize(st));  // the host vectors above must outlive the copies
  D->since_build = 0;
  D->rebuild_next = false;
}

void md_set_barostat(e3mi_md* D, double pressure_bar, int interval, double fraction, const double* dv_max,
                     const uint64_t* seeds, const int64_t* move0) {
  E3MI_REQUIRE(interval >= 0, E3MI_EINVAL, "interval must be >= 0");
  if (interval == 0) {
    D->baro_interval = 0;
    return;
  }
  E3MI_REQUIRE(D->gamma > 0 && D->temperature > 0, E3MI_EINVAL,
               "the barostat needs Langevin dynamics at a positive temperature (e3mi_md_set_langevin)");
  E3MI_REQUIRE(std::isfinite(pressure_bar), E3MI_EINVAL, "pressure must be finite");
  E3MI_REQUIRE(dv_max || (fraction > 0 && fraction < 1), E3MI_EINVAL, "volume fraction must be in (0, 1)");
  e3mi_graph* G = D->graph;
  D->dv_max.assign(D->S, 0.0);
  D->baro_seed.assign(D->S, 0);
  D->baro_move.assign(D->S, 0);
  for (int s = 0; s < D->S; ++s) {
    for (int k = 0; k < 3; ++k)
      E3MI_REQUIRE(D->pbc_h[3 * s + k], E3MI_EINVAL, "the barostat needs structures periodic along every axis");
    D->dv_max[s] = dv_max ? dv_max[s] : fraction * G->box_h[3 * s] * G->box_h[3 * s + 1] * G->box_h[3 * s + 2];
    E3MI_REQUIRE(std::isfinite(D->dv_max[s]) && D->dv_max[s] > 0, E3MI_EINVAL, "volume steps must be positive");
    D->baro_seed[s] = seeds ? seeds[s] : (uint64_t)s;
    D->baro_move[s] = move0 ? move0[s] : 0;
    E3MI_REQUIRE(D->baro_move[s] >= 0, E3MI_EINVAL, "move counters must be >= 0");
  }
  D->pressure_bar = pressure_bar;
  D->baro_interval = interval;
}

void md_set_langevin(e3mi_md* D, double temperature, double gamma, const uint64_t* seeds, const int64_t* step0,
                     hipStream_t st) {
  E3MI_REQUIRE(std::isfinite(temperature) && temperature >= 0, E3MI_EINVAL, "temperature must be >= 0");
  E3MI_REQUIRE(std::isfinite(gamma) && gamma >= 0, E3MI_EINVAL, "friction must be >= 0");
  Allocator* a = &D->model->alloc;
  std::vector<uint64_t> sd((size_t)D->S);
  std::vector<int64_t> s0((size_t)D->S);
  for (int s = 0; s < D->S; ++s) {
    sd[s] = seeds ? seeds[s] : (uint64_t)s;
    s0[s] = step0 ? step0[s] : 0;
    E3MI_REQUIRE(s0[s] >= 0, E3MI_EINVAL, "step offsets must be >= 0");
  }
  // the step offset is relative to this object's own step count
  for (int s = 0; s < D->S; ++s) s0[s] -= D->steps;
  D->step0_h = s0;
  E3MI_HIP(hipStreamSynchronize(st));
  D->seeds = upload(a, sd.data(), sizeof(uint64_t) * sd.size());
  D->step0 = upload(a, s0.data(), sizeof(int64_t) * s0.size());
  D->temperature = temperature;
  D->gamma = gamma;
}

void set_error(const std::string& m) { g_last_error = m; }

}  // namespace
}  // namespace e3mi

// ---- evaluation without allocation ----------------------------------------------------
// Per-call workspace for callers that cannot allocate: a static device array,
// held by every GPU the library runs on until the process ends. Host code uses
// its device address (from hipGetSymbolAddress, per device), never its name.
constexpr size_t kStaticScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace e3mi {
namespace {

std::mutex g_scratch_mu;
std::array<char*, 64> g_scratch_ptr{};

// the array's address on the current device (looked up once per device)
char* static_scratch() {
  int dev = 0;
  E3MI_HIP(hipGetDevice(&dev));
  E3MI_REQUIRE(dev >= 0 && dev < (int)g_scratch_ptr.size(), E3MI_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    E3MI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    E3MI_REQUIRE(p != nullptr, E3MI_EDEVICE, "static scratch has no device address");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  return g_scratch_ptr[dev];
}

// energy_forces with every workspace buffer carved from the static scratch:
// the model's own workspace and allocator are set aside for the call and put
// back afterwards (also on error).
void energy_forces_static(e3mi_model* M, e3mi_graph* G, const double* pos, double* energy, float* forces,
                          double* atom_energy, hipStream_t st) {
  // layers with per-edge R must hold every edge's R at once (receiver chunks
  // read the row pointer back to the host)
  for (int t = 1; t <= M->cfg.layers; ++t) {
    const LayerPlan& L = M->plans[t - 1];
    if ((t == 1 && factorised_first(M)) || fused_last(M, L, false, M->precision == E3MI_BF16_MIX)) continue;
    E3MI_REQUIRE(r_chunk_edges(M, G->E, L.p_used * M->cfg.channels) >= (size_t)(G->E + 1), E3MI_EINVAL,
                 "the per-edge radial weights of every edge must fit the model's R budget at once");
  }
  char* base = static_scratch();
  Workspace saved = std::move(M->ws);
  const Allocator saved_alloc = M->alloc;
  const bool prof_on = M->prof.on;
  M->ws = Workspace{};
  M->alloc.arena = base;
  M->alloc.arena_bytes = kStaticScratchBytes;
  M->alloc.arena_used = 0;
  M->prof.on = false;  // timing events are not allocated either
  auto restore = [&] {
    M->ws = Workspace{};  // the carved buffers are released while the arena is in place (no frees)
    M->alloc = saved_alloc;
    M->ws = std::move(saved);
    M->prof.on = prof_on;
  };
  try {
    energy_forces(M, G, pos, energy, forces, atom_energy, st);
  } catch (...) {
    restore();
    throw;
  }
  restore();
}

}  // namespace
}  // namespace e3mi

// ---- C ABI -----------------------------------------------------------------------------------

#define E3MI_API_BEGIN \
  e3mi::set_error(""); \
  try {
#define E3MI_API_END                                  \
  }                                                   \
  catch (const e3mi::Error& e) {                      \
    e3mi::set_error(e.what());                        \
    return e.code;                                    \
  }                                                   \
  catch (const std::bad_alloc&) {                     \
    e3mi::set_error("host allocation failed");        \
    return E3MI_ENOMEM;                               \
  }                                                   \
  catch (const std::exception& e) {                   \
    e3mi::set_error(e.what());                        \
    return E3MI_EINVAL;                               \
  }                                                   \
  return E3MI_OK;

extern "C" {

int e3mi_weight_count(const char* config_json, size_t* n_weights) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(n_weights, E3MI_EINVAL, "null output");
  *n_weights = e3mi::weight_count(e3mi::parse_config(config_json));
  E3MI_API_END
}

int e3mi_model_create(const char* config_json, const double* weights_host, size_t n_weights, int precision,
                      e3mi_alloc_fn alloc, e3mi_free_fn free_fn, void* ctx, e3mi_model** out) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(out, E3MI_EINVAL, "null output");
  *out = nullptr;
  *out = e3mi::new_model(config_json, weights_host, n_weights, precision, alloc, free_fn, ctx);
  E3MI_API_END
}

int e3mi_model_destroy(e3mi_model* model) {
  E3MI_API_BEGIN
  delete model;
  E3MI_API_END
}

int e3mi_build_graph(e3mi_model* model, int n_structures, const int64_t* atom_offsets, const double* pos,
                     const int32_t* species, const double* cell, const uint8_t* pbc, double cutoff, double skin,
                     void* stream, e3mi_graph** out) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(out, E3MI_EINVAL, "null output");
  *out = nullptr;
  *out = e3mi::new_graph(model, n_structures, atom_offsets, pos, species, cell, pbc, cutoff, skin,
                         e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_graph_destroy(e3mi_graph* graph) {
  E3MI_API_BEGIN
  delete graph;
  E3MI_API_END
}

int e3mi_graph_info(const e3mi_graph* graph, int64_t* n_atoms, int64_t* n_skin_edges) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(graph, E3MI_EINVAL, "null graph");
  if (n_atoms) *n_atoms = graph->N;
  if (n_skin_edges) *n_skin_edges = graph->E;
  E3MI_API_END
}

int e3mi_graph_copy_edges(const e3mi_graph* graph, int32_t* row_ptr, int32_t* src, int32_t* shift, int32_t* rev,
                          void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(graph, E3MI_EINVAL, "null graph");
  hipStream_t st = e3mi::as_stream(stream);
  const size_t E = (size_t)graph->E, N = (size_t)graph->N;
  if (row_ptr)
    E3MI_HIP(hipMemcpyAsync(row_ptr, graph->row_ptr->p, sizeof(int) * (N + 1), hipMemcpyDeviceToDevice, st));
  if (src && E) E3MI_HIP(hipMemcpyAsync(src, graph->src->p, sizeof(int) * E, hipMemcpyDeviceToDevice, st));
  if (rev && E) E3MI_HIP(hipMemcpyAsync(rev, graph->rev->p, sizeof(int) * E, hipMemcpyDeviceToDevice, st));
  if (shift) e3mi::launch_unpack_shift(graph->shift->as<int>(), (int)E, shift, st);
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_energy_forces(e3mi_model* model, e3mi_graph* graph, const double* pos, double* energy, float* forces,
                       double* atom_energy, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model && graph && energy && forces, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(graph->model == model, E3MI_EINVAL, "graph was built for another model");
  E3MI_REQUIRE(graph->N == 0 || pos, E3MI_EINVAL, "null positions");
  e3mi::energy_forces(model, graph, pos, energy, forces, atom_energy, e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_energy_forces_static(e3mi_model* model, e3mi_graph* graph, const double* pos, double* energy,
                              float* forces, double* atom_energy, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model && graph && energy && forces, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(graph->model == model, E3MI_EINVAL, "graph was built for another model");
  E3MI_REQUIRE(graph->N == 0 || pos, E3MI_EINVAL, "null positions");
  e3mi::energy_forces_static(model, graph, pos, energy, forces, atom_energy, e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_param_grad(e3mi_model* model, e3mi_graph* graph, const double* pos, const double* grad_energy,
                    const float* grad_forces, double* grad_weights, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model && graph && grad_energy && grad_forces && grad_weights, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(graph->model == model, E3MI_EINVAL, "graph was built for another model");
  E3MI_REQUIRE(graph->N == 0 || pos, E3MI_EINVAL, "null positions");
  e3mi::param_grad(model, graph, pos, grad_energy, grad_forces, grad_weights, e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_hessian_vector(e3mi_model* model, e3mi_graph* graph, const double* pos, const float* v, float* hv,
                        void* stream) {
  return e3mi_hessian_vectors(model, graph, pos, 1, v, hv, stream);
}

int e3mi_hessian_vectors(e3mi_model* model, e3mi_graph* graph, const double* pos, int n_vec, const float* v,
                         float* hv, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model && graph, E3MI_EINVAL, "null argument");
  E3MI_REQUIRE(graph->model == model, E3MI_EINVAL, "graph was built for another model");
  E3MI_REQUIRE(graph->N == 0 || n_vec == 0 || (pos && v && hv), E3MI_EINVAL, "null positions, vectors or output");
  if (graph->N) e3mi::hessian_vectors(model, graph, pos, n_vec, v, hv, e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_model_set_r_chunk_bytes(e3mi_model* model, size_t bytes) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model, E3MI_EINVAL, "null model");
  E3MI_REQUIRE(bytes >= (size_t)1 << 20, E3MI_EINVAL, "the R chunk must be at least 1 MiB");
  model->r_chunk_bytes = bytes;
  E3MI_API_END
}

int e3mi_model_set_r_keep_bytes(e3mi_model* model, size_t bytes) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model, E3MI_EINVAL, "null model");
  model->r_keep_bytes = bytes;
  E3MI_API_END
}

int e3mi_model_set_flags(e3mi_model* model, int flags) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model, E3MI_EINVAL, "null model");
  E3MI_REQUIRE((flags & ~15) == 0, E3MI_EINVAL, "unknown flag");
  model->first_factorised = (flags & 1) == 0;
  model->last_fused = (flags & 4) != 0 && (flags & 2) == 0;
  model->edge_pairs = (flags & 8) == 0;
  E3MI_API_END
}

int e3mi_model_set_weights(e3mi_model* model, const double* weights_host, size_t n_weights) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model, E3MI_EINVAL, "null model");
  e3mi::set_weights(model, weights_host, n_weights);
  E3MI_API_END
}

int e3mi_graph_last_edge_count(const e3mi_graph* graph, int64_t* n_edges, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(graph && n_edges, E3MI_EINVAL, "null argument");
  int e = 0;
  if (graph->N) {
    hipStream_t st = e3mi::as_stream(stream);
    E3MI_HIP(hipMemcpyAsync(&e, graph->row_ptr_x->as<int>() + graph->N, sizeof(int), hipMemcpyDeviceToHost, st));
    E3MI_HIP(hipStreamSynchronize(st));
  }
  *n_edges = e;
  E3MI_API_END
}

int e3mi_md_create(e3mi_model* model, int n_structures, const int64_t* atom_offsets, const double* pos,
                   const double* vel, const int32_t* species, const double* masses, const double* cell,
                   const uint8_t* pbc, double cutoff, double skin, int rebuild_every, void* stream, e3mi_md** out) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(out, E3MI_EINVAL, "null output");
  *out = nullptr;
  *out = e3mi::new_md(model, n_structures, atom_offsets, pos, vel, species, masses, cell, pbc, cutoff, skin,
                      rebuild_every, e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_md_step(e3mi_md* md, int n_steps, double dt_fs, double* energy_out, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  e3mi::md_step(md, n_steps, dt_fs, energy_out, e3mi::as_stream(stream));
  E3MI_HIP(hipGetLastError());
  E3MI_API_END
}

int e3mi_md_state(const e3mi_md* md, double* pos, double* vel, float* forces, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  hipStream_t st = e3mi::as_stream(stream);
  const size_t n = (size_t)md->N;
  if (n && pos) E3MI_HIP(hipMemcpyAsync(pos, md->x->p, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  if (n && vel) E3MI_HIP(hipMemcpyAsync(vel, md->v->p, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice, st));
  if (n && forces) E3MI_HIP(hipMemcpyAsync(forces, md->F->p, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, st));
  E3MI_API_END
}

int e3mi_md_stats(const e3mi_md* md, int64_t* steps, int64_t* rebuilds, int64_t* skin_violations) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  if (steps) *steps = md->steps;
  if (rebuilds) *rebuilds = md->rebuilds;
  if (skin_violations) *skin_violations = md->skin_violations;
  E3MI_API_END
}

int e3mi_md_set_langevin(e3mi_md* md, double temperature_K, double friction_per_fs, const uint64_t* seeds,
                         const int64_t* step0, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  e3mi::md_set_langevin(md, temperature_K, friction_per_fs, seeds, step0, e3mi::as_stream(stream));
  E3MI_API_END
}

int e3mi_md_set_barostat(e3mi_md* md, double pressure_bar, int interval, double volume_fraction,
                         const double* dv_max, const uint64_t* seeds, const int64_t* move0) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  e3mi::md_set_barostat(md, pressure_bar, interval, volume_fraction, dv_max, seeds, move0);
  E3MI_API_END
}

int e3mi_md_cells(const e3mi_md* md, double* cells, int64_t* proposed, int64_t* accepted) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  if (cells) std::memcpy(cells, md->cell_h.data(), sizeof(double) * 9 * md->S);
  if (proposed) *proposed = md->baro_proposed;
  if (accepted) *accepted = md->baro_accepted;
  E3MI_API_END
}

int e3mi_graph_set_total_charge(e3mi_graph* graph, const double* total_charge) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(graph && total_charge, E3MI_EINVAL, "null argument");
  for (int s = 0; s < graph->S; ++s)
    E3MI_REQUIRE(std::isfinite(total_charge[s]), E3MI_EINVAL, "total charges must be finite");
  E3MI_HIP(hipMemcpy(graph->charge->p, total_charge, sizeof(double) * graph->S, hipMemcpyHostToDevice));
  E3MI_API_END
}

int e3mi_md_set_total_charge(e3mi_md* md, const double* total_charge, void* stream) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(md, E3MI_EINVAL, "null md");
  const int rc = e3mi_graph_set_total_charge(md->graph, total_charge);
  if (rc != E3MI_OK) return rc;
  hipStream_t st = e3mi::as_stream(stream);
  e3mi::energy_forces(md->model, md->graph, md->x->as<double>(), md->energy->as<double>(), md->F->as<float>(),
                      nullptr, st);
  E3MI_HIP(hipStreamSynchronize(st));
  E3MI_API_END
}

int e3mi_md_destroy(e3mi_md* md) {
  E3MI_API_BEGIN
  if (md) delete md->graph;
  delete md;
  E3MI_API_END
}

size_t e3mi_footprint_bytes(const e3mi_model* model, int64_t n_atoms, int64_t n_edges) {
  if (!model) return 0;
  return e3mi::footprint(model, n_atoms, n_edges);
}

int e3mi_profile_enable(e3mi_model* model, int enable) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model, E3MI_EINVAL, "null model");
  if (enable) model->prof.reset();
  model->prof.on = enable != 0;
  E3MI_API_END
}

int e3mi_profile_select(e3mi_model* model, const char* stage) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model, E3MI_EINVAL, "null model");
  model->prof.only_stage = model->prof.only_layer = -1;
  if (stage && *stage) {
    int layer = -1;
    model->prof.only_stage = e3mi::parse_stage(stage, &layer);
    model->prof.only_layer = layer;
  }
  E3MI_API_END
}

int e3mi_profile_query(e3mi_model* model, const char* stage, double* total_ms, int64_t* launches) {
  E3MI_API_BEGIN
  E3MI_REQUIRE(model && stage && total_ms && launches, E3MI_EINVAL, "null argument");
  model->prof.drain();
  int layer = -1;
  const int sid = e3mi::parse_stage(stage, &layer);
  double ms = 0.0;
  int64_t n = 0;
  for (int l = 0; l < 8; ++l) {
    if (layer >= 0 && l != layer) continue;
    const size_t idx = (size_t)sid * 8 + l;
    if (idx < model->prof.ms.size()) {
      ms += model->prof.ms[idx];
      n += model->prof.count[idx];
    }
  }
  *total_ms = ms;
  *launches = n;
  E3MI_API_END
}

const char* e3mi_last_error(void) { return e3mi::g_last_error.c_str(); }

}  // extern "C"
