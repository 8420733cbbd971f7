/*
 * e3mi — equivariant message-passing interaction on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library. It evaluates the energy and forces of an equivariant
 * interatomic potential whose hot loop is the Clebsch-Gordan tensor product
 * that the paper's backend accelerates (Section 4, "Accelerating equivariant
 * operations"; Appendix F, MACE and NequIP hyperparameter tables), and runs
 * velocity-Verlet molecular dynamics on it (Section 1: batched MD; Appendix H,
 * table of ms per MD step).
 *
 * Problem statement (Section 3.2 and Appendix A: a chemical system — positions,
 * atomic numbers, cell — is turned into a graph with a cutoff radius and the
 * force field returns its energy, with forces by default): several structures
 * are packed along the atom axis by `atom_offsets`; structure s owns atoms
 * atom_offsets[s] .. atom_offsets[s+1]-1.
 *
 * Units: angstrom, eV, fs, amu. Forces are -dE/dr (Section 5.2 defines the
 * Hessian as minus the derivative of the forces, i.e. forces are -dE/dr).
 *
 * Conventions shared by every entry point:
 *  - Pointers documented as "device" must be device (HBM) addresses; "host"
 *    pointers are ordinary CPU memory read during the call only.
 *  - The caller owns every array it passes. The library owns the opaque
 *    handles and their device buffers, obtained from the allocator given at
 *    e3mi_model_create (or hipMalloc when none is given).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    Outputs are valid once the stream has been synchronised. Calls that
 *    must learn a size from the device (graph building) synchronise the
 *    stream themselves, as documented.
 *  - A model handle holds one scratch workspace: calls that use the same
 *    model must be ordered (same stream, or externally synchronised).
 *  - Every function returns an e3mi_status. No exception crosses the ABI.
 *    On error, outputs are unspecified, handles stay valid, and
 *    e3mi_last_error() describes the failure (thread-local).
 */
#ifndef E3MI_H
#define E3MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct e3mi_model e3mi_model; /* weights + workspace */
typedef struct e3mi_graph e3mi_graph; /* neighbour lists of a packed batch */
typedef struct e3mi_md e3mi_md;       /* MD state: x, v (FP64), forces, graph */

typedef enum e3mi_status {
  E3MI_OK = 0,
  E3MI_EINVAL = -1,      /* bad argument (null pointer, inconsistent sizes, bad config) */
  E3MI_ENOMEM = -2,      /* the allocator returned NULL */
  E3MI_EDEVICE = -3,     /* a HIP runtime call failed */
  E3MI_EOVERFLOW = -4,   /* an image index or an edge count does not fit its type */
  E3MI_ENAN = -5,        /* non-finite positions or energies */
  E3MI_EUNSUPPORTED = -6 /* valid input the library does not handle (e.g. triclinic cell) */
} e3mi_status;

typedef enum e3mi_precision {
  E3MI_FP32 = 0,    /* every contraction in FP32 */
  E3MI_BF16_MIX = 1 /* radial-MLP and channel-mix GEMM inputs rounded to BF16, FP32 accumulation;
                       tensor product FP32; energy reduction and MD update FP64 */
} e3mi_precision;

/* Device allocator callbacks: alloc returns `bytes` of device memory aligned to
 * 256 bytes, or NULL; free releases a pointer alloc returned. */
typedef void* (*e3mi_alloc_fn)(size_t bytes, void* ctx);
typedef void (*e3mi_free_fn)(void* ptr, void* ctx);

/* Model configuration (JSON object; all keys required unless marked optional):
 *   lmax (2 or 3), channels (C: 32, 64 or 128), layers (1 <= T <= 8),
 *   n_species, cutoff (r_c, angstrom), avg_neighbors (nu, the constant the
 *   neighbour sum is divided by), n_basis (8), envelope_p, radial_hidden (64),
 *   readout_hidden (16);
 *   coulomb (optional JSON boolean, default false) and, when true,
 *   soft_core_r0 (r0 > 0, angstrom): Section 5.1 electrostatics. A linear
 *   charge head on the last layer's scalar features gives q_i = w_q . h_i +
 *   b_q[z_i]; the charge-correction equation shifts the charges of each
 *   structure uniformly so that they sum to its total charge Q_s (0 unless
 *   set by e3mi_graph_set_total_charge); the long-range-interaction equation
 *   adds 1/2 sum_{i != j in s} k_e q~_i q~_j / chi(r_ij) over ALL pairs of a
 *   structure (no cutoff), with PhysNet's soft core 1/chi(r) = f(r/r0) /
 *   sqrt(r^2 + 1) + (1 - f(r/r0)) / r, f(x) = 1 - 6x^5 + 15x^4 - 10x^3 on
 *   [0, 1) and 0 beyond, k_e = 14.3996 eV A. Each atom's energy carries half
 *   of each of its pair terms. Open structures only: building a graph with a
 *   periodic axis for such a model fails with E3MI_EUNSUPPORTED, and so does
 *   e3mi_param_grad;
 *   correlation (optional, 1 or 2, default 1): 2 inserts MACE's product block
 *   of body order 2 (Appendix F: the MACE models use correlation 2) in every
 *   layer. With A~^l the layer's channel mix (no self connection) for every
 *   order l <= lmax, per atom of species z and channel k:
 *     B^L = w1[z, L] A~^L + sum_p w2[z, p] (A~^{l1} (x) A~^{l2})_L
 *   over the couplings p = (l1 <= l2, L) of the CG table (natural parity,
 *   ordered by L, then l1, then l2; L <= lmax, only L = 0 in the last layer),
 *   then h~^L = B^L W_lin,L + h_in^L W_self,L and the gate. Every layer then
 *   computes every order of A (no fused scalar-only last layer). The
 *   second-order passes (e3mi_param_grad, e3mi_hessian_vector) carry the
 *   block's tangent B_dot = f'(A~) A~_dot and its reverse.
 * Readings of the paper behind each key: Appendix F tables (l_max, channels,
 * layers, num_rbf 8, radial net of 2 hidden layers of 64 with swish,
 * polynomial envelope, gate nonlinearity, readout 16x0e -> 0e, cutoff 5 A).
 *
 * Weights: one host FP64 vector, row-major tensors concatenated in this order
 * (P_t = number of natural-parity paths (l1,l2,l3) of layer t, ordered by
 * (l3, l1, l2); l1 runs over the layer's input orders — {0} for t = 1,
 * 0..lmax after — and l2, l3 over 0..lmax; P_{t,l3} those with output l3):
 *   emb [n_species, C]
 *   for t = 1..T: rad1 [n_basis, H], rad2 [H, H], rad3 [H, P_t*C] (column p*C + k),
 *                 mix_l3 [P_{t,l3}*C, C] for l3 = 0..lmax (row q*C + k),
 *                 self_l3 [C, C] for each l3 among the layer's input orders,
 *                 with correlation 2 (Lo = 0 for t = T, else lmax; n_p couplings):
 *                 sym1 [n_species, Lo+1, C], sym2 [n_species, n_p, C], lin_L [C, C] for L = 0..Lo
 *   read1 [C, readout_hidden], read2 [readout_hidden, 1], e0 [n_species]
 *   with coulomb: qhead [C], qbias [n_species]
 */

/* Number of FP64 weights the configuration expects. */
int e3mi_weight_count(const char* config_json, size_t* n_weights);

/* Create a model. weights_host: n_weights FP64 values (host). precision: an
 * e3mi_precision. alloc/free may be NULL (then hipMalloc/hipFree are used);
 * ctx is passed to them unchanged. Synchronous (uploads weights). */
int e3mi_model_create(const char* config_json, const double* weights_host, size_t n_weights,
                      int precision, e3mi_alloc_fn alloc, e3mi_free_fn free_fn, void* ctx,
                      e3mi_model** out);
int e3mi_model_destroy(e3mi_model* model);

/* Build the neighbour lists of a packed batch (Section 3.2: graph from a
 * chemical system and a cutoff radius). Lists every directed edge i <- j with
 * integer image vector n (zero along non-periodic axes) such that
 *   0 < |r_j - r_i + n . cell| < cutoff + skin,
 * per structure (edges never join structures), stored in CSR by receiver i and
 * sorted by (j, n) within a receiver; each edge knows its reverse (j <- i, -n).
 *   n_structures   S >= 1
 *   atom_offsets   host int64 [S+1], non-decreasing, atom_offsets[0] = 0
 *   pos            device FP64 [N, 3]
 *   species        device int32 [N], values in [0, n_species) (EINVAL otherwise)
 *   cell           host FP64 [S, 3, 3], rows are lattice vectors; must be
 *                  diagonal (orthorhombic) on periodic axes, else EUNSUPPORTED
 *   pbc            host uint8 [S, 3], periodic flags
 *   cutoff         >= the model's cutoff; skin >= 0
 * Synchronises `stream` twice (to size the cell grid and the edge arrays).
 * The graph stays valid while every atom stays within skin/2 of its position
 * at build time; energy_forces re-selects the edges inside the model cutoff on
 * every call. */
int e3mi_build_graph(e3mi_model* model, int n_structures, const int64_t* atom_offsets,
                     const double* pos, const int32_t* species, const double* cell,
                     const uint8_t* pbc, double cutoff, double skin, void* stream,
                     e3mi_graph** out);
int e3mi_graph_destroy(e3mi_graph* graph);

/* Sizes of a graph: atoms N and edges of the skin list. */
int e3mi_graph_info(const e3mi_graph* graph, int64_t* n_atoms, int64_t* n_skin_edges);

/* Copy the skin neighbour list to caller device buffers: row_ptr int32 [N+1],
 * src int32 [E], shift int32 [E, 3] (image vector n), rev int32 [E] (index of
 * the reverse edge). Any output may be NULL. Asynchronous on `stream`. */
int e3mi_graph_copy_edges(const e3mi_graph* graph, int32_t* row_ptr, int32_t* src, int32_t* shift,
                          int32_t* rev, void* stream);

/* Energy and forces of every structure (Section 4 hot path; Section 5.3 readout
 * E = sum_i [R(h_i) + E0(z_i)] with one head). pos: device FP64 [N, 3] (the
 * same atoms as the graph). energy: device FP64 [S] (per-structure sums in a
 * fixed order). forces: device FP32 [N, 3]. atom_energy: device FP64 [N] or
 * NULL. Asynchronous on `stream`. */
int e3mi_energy_forces(e3mi_model* model, e3mi_graph* graph, const double* pos, double* energy,
                       float* forces, double* atom_energy, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation as e3mi_energy_forces, same arguments and results, with every
 * per-call workspace buffer taken from a static device array of
 * E3MI_STATIC_SCRATCH_BYTES (128 MiB) that the library holds on each GPU it
 * runs on until the process ends. Calls no device allocator (the model's
 * allocator callbacks included) and clears memory with kernels, not memsets.
 * The graph must have been built beforehand (e3mi_build_graph allocates).
 * Errors: ENOMEM when the evaluation needs more than the array (outputs are
 * then unspecified; roughly N x 16 x C x 4 bytes per feature buffer plus
 * 4 x P x C bytes per edge for each layer's radial weights and their adjoint),
 * EINVAL when a layer's per-edge radial weights would have to be split into
 * receiver chunks. The array keeps the last call's contents; every buffer the
 * evaluation reads is written first. All calls on one GPU share the array:
 * calls that overlap in time on one GPU race, so issue them in order on one
 * stream. The model's own workspace is left as it was. */
#define E3MI_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
int e3mi_energy_forces_static(e3mi_model* model, e3mi_graph* graph, const double* pos, double* energy,
                              float* forces, double* atom_energy, void* stream);

/* Gradient of a loss L(E, F) with respect to the weights, given the upstream
 * gradients grad_energy = dL/dE (device FP64 [S]) and grad_forces = dL/dF
 * (device FP32 [N, 3]): writes dL/dtheta = sum_s dL/dE_s dE_s/dtheta +
 * sum_i dL/dF_i . dF_i/dtheta to grad_weights (device FP64, n_weights, the
 * layout of the weight vector; entries the energy does not depend on are 0).
 * Training on energies and forces (Appendix F recipe; §5.2 differentiates
 * forces for Hessian-row labels) needs this second-order term: it is formed
 * as minus the weight gradient of the directional derivative of E along
 * dL/dF, by a tangent pass and a reverse pass over primal and tangent values.
 * Recomputes the forward pass; does not need a preceding energy_forces call.
 * Asynchronous on `stream`. */
int e3mi_param_grad(e3mi_model* model, e3mi_graph* graph, const double* pos, const double* grad_energy,
                    const float* grad_forces, double* grad_weights, void* stream);

/* Hessian-vector product of the energy with respect to the positions
 * (Section 5.2, the full-Hessian equation): hv_j = sum_i H_ji v_i with
 * H_ij = d^2 E / dr_i dr_j = -dF_i/dr_j, summed over the structures of the
 * graph (structures do not interact, so H is block diagonal). v and hv:
 * device FP32 [N, 3] (hv is overwritten). A sampled Hessian row of the
 * paper's training scheme is hv for v = one unit vector per structure (atom
 * i_s, Cartesian axis a); the full Hessian of a batch takes 3 max_s N_s
 * products. Computed like e3mi_param_grad (tangent pass along v, reverse
 * pass over primal and tangent values) with the reverse pass continued
 * through every layer's harmonics and radial basis to the positions; no
 * weight gradients are formed. Errors: E3MI_EUNSUPPORTED for models with the
 * Coulomb term. Asynchronous on `stream`. */
int e3mi_hessian_vector(e3mi_model* model, e3mi_graph* graph, const double* pos, const float* v, float* hv,
                        void* stream);

/* n_vec Hessian-vector products at the same positions: v and hv are device
 * FP32 [n_vec, N, 3]; hv[k] = H v[k]. The primal forward pass runs once and
 * each direction costs one tangent and one reverse pass. Same errors as
 * e3mi_hessian_vector. */
int e3mi_hessian_vectors(e3mi_model* model, e3mi_graph* graph, const double* pos, int n_vec, const float* v,
                         float* hv, void* stream);

/* Evaluation options of a model (bit mask, default 0):
 *   E3MI_FLAG_UNFACTORISED_FIRST_LAYER (1): evaluate the first layer like
 *     the others (per-edge radial weights R and tensor product) instead of
 *     the exact species factorisation of its neighbour sum (its input is the
 *     embedding of the sender's species); results agree to rounding. */
#define E3MI_FLAG_UNFACTORISED_FIRST_LAYER 1
/*   The last layer (scalar outputs only: Section 4's tensor product
 *     restricted to the paths that reach the energy) has two evaluations
 *     whose results agree to rounding. By default it keeps per-edge radial
 *     weights R in memory and runs separate radial / tensor-product kernels
 *     (measured faster on MI355X).
 *   E3MI_FLAG_FUSED_LAST_LAYER (4) selects the fused kernels instead. They
 *     never store R: the neighbour sum is taken as W3^T times a per-receiver
 *     product of hidden activations and contracted features. They are used
 *     only in FP32 with two or more layers; the parameter-gradient pass
 *     always uses the per-edge form.
 *   E3MI_FLAG_UNFUSED_LAST_LAYER (2) forces the per-edge form even when bit
 *     4 is set. */
#define E3MI_FLAG_UNFUSED_LAST_LAYER 2
#define E3MI_FLAG_FUSED_LAST_LAYER 4
/*   An edge and its reverse have exactly opposite vectors (the same FP64
 *     difference of the two positions plus the image shift, negated), so
 *     equal lengths and equal radial weights R. By default a layer whose
 *     edges are all in memory at once (one receiver chunk) runs its radial
 *     MLP once per edge pair. In an energy+forces call it stores R once per
 *     pair (the same values as edge by edge; the second-order passes write
 *     them to both edges' rows). Its adjoint runs once per pair on the sum of
 *     the two edges' dR (forces agree with the edge-by-edge adjoint to
 *     rounding). The species-factorised first layer's radial hidden layers
 *     run once per pair likewise.
 *   E3MI_FLAG_RADIAL_PER_EDGE (8) runs all of them per edge instead, as
 *     layers in receiver chunks always do; results are then bitwise those of
 *     any chunking. */
#define E3MI_FLAG_RADIAL_PER_EDGE 8
int e3mi_model_set_flags(e3mi_model* model, int flags);

/* Most bytes of per-edge radial weights R (and of their adjoint) that an
 * energy_forces call holds at once for the layers evaluated with R in memory
 * (middle layers, and every layer of a model with the product block); default
 * 8 GiB, at least 1 MiB. Larger edge sets are processed in chunks of whole
 * receivers (the adjoint then recomputes R per chunk), so a 100,000-atom,
 * 9-million-edge, 3-layer model (about 106 GB of R per layer in FP32, Section
 * 4's tensor product at scale) runs in bounded memory. The chunking reads the
 * pruned row pointer back to the host once per call. Chunked layers run the
 * radial MLP edge by edge; results are bitwise those of the unchunked
 * evaluation with E3MI_FLAG_RADIAL_PER_EDGE (each receiver's and each
 * sender's sums run in the same order whatever the chunks), and agree with
 * the default per-pair radial adjoint of an unchunked layer to rounding. */
int e3mi_model_set_r_chunk_bytes(e3mi_model* model, size_t bytes);

/* Most bytes of per-edge R kept for every edge inside the cutoff, summed
 * over the layers evaluated in receiver chunks (default 160 GiB of the 288 GB
 * of HBM; 0: never). Layers are taken in order while the sum fits; such a layer's
 * forward pass writes every chunk's R into one buffer and its adjoint reads
 * it there instead of recomputing R chunk by chunk (dR and the sender
 * messages stay chunk-sized). Results are bitwise the same either way. */
int e3mi_model_set_r_keep_bytes(e3mi_model* model, size_t bytes);

/* Replace the weights (host FP64, same configuration and layout as at
 * creation), e.g. after an optimiser step. Synchronises the device first. */
int e3mi_model_set_weights(e3mi_model* model, const double* weights_host, size_t n_weights);

/* Number of edges inside the model cutoff at the last energy_forces call on
 * this graph. Synchronises `stream`. */
int e3mi_graph_last_edge_count(const e3mi_graph* graph, int64_t* n_edges, void* stream);

/* Total charge Q_s of every structure (host FP64 [S], elementary charges) for
 * the charge correction of Section 5.1; used by models with the Coulomb term,
 * ignored by others. A new graph starts neutral. Synchronous. */
int e3mi_graph_set_total_charge(e3mi_graph* graph, const double* total_charge);

/* Velocity-Verlet NVE molecular dynamics on a packed batch (Section 1: batched
 * MD; Appendix H: ms per MD step). The state (positions and velocities in
 * FP64, forces, neighbour lists) stays on the device. Inputs as for
 * e3mi_build_graph plus: vel device FP64 [N, 3] (angstrom/fs), masses host
 * FP64 [n_species] (amu), rebuild_every >= 1 (steps between neighbour
 * rebuilds). Positions are kept as integrated (never wrapped; image indices
 * must stay within +-127 cells, else EOVERFLOW at the next rebuild). The lists
 * are rebuilt every rebuild_every steps, and early on any step whose drift
 * takes an atom more than skin/2 from its position at the last build (counted
 * as a skin violation): that step's force evaluation and final kick are redone
 * on the new lists, so every step's forces see every pair inside the cutoff.
 * To keep redone steps rare, each drift also forecasts the largest
 * displacement after the next drift (|x - x_build| + dt |v|); when that
 * reaches skin/2 the next step rebuilds before its force evaluation.
 * pos/vel are copied; the caller's buffers are not referenced afterwards.
 * Synchronises `stream`. */
int e3mi_md_create(e3mi_model* model, int n_structures, const int64_t* atom_offsets,
                   const double* pos, const double* vel, const int32_t* species,
                   const double* masses, const double* cell, const uint8_t* pbc, double cutoff,
                   double skin, int rebuild_every, void* stream, e3mi_md** out);

/* Advance n_steps steps of dt_fs:
 *   v += dt/2 * kappa F/m;  x += dt v;  F = F(x);  v += dt/2 * kappa F/m
 * with kappa = 0.009648533 A/fs^2 per (eV/A)/amu, positions and velocities in
 * FP64. energy_out: device FP64 [S], potential energy after the last step, or
 * NULL. Synchronises `stream` when a neighbour rebuild is due (every
 * rebuild_every steps); on the other steps the host waits until the device has
 * done the step's drift (to check the skin, above), while the step's force
 * evaluation stays queued. */
int e3mi_md_step(e3mi_md* md, int n_steps, double dt_fs, double* energy_out, void* stream);

/* Switch the integrator to Langevin dynamics (Section 5.5: the NVT
 * integrator; batched systems with independent random seeds), BAOAB
 * splitting per step:
 *   v += dt/2 kappa F/m;  x += dt/2 v;
 *   v = c1 v + sqrt(1 - c1^2) sqrt(kB T kappa / m) z,  c1 = exp(-friction dt);
 *   x += dt/2 v;  F = F(x);  v += dt/2 kappa F/m
 * temperature_K >= 0, friction_per_fs >= 0 (0 returns to velocity Verlet).
 * z: three standard normals per atom from Philox4x64-10 (Salmon et al.,
 * SC'11) with key (seeds[s], 0) and counter (step, index of the atom in its
 * structure s, 0, 0), Box-Muller on the uniforms ((x >> 11) + 1/2) 2^-53.
 * seeds: host uint64 [S] (NULL: s); step0: host int64 [S], the counter of
 * each structure's next step (NULL: 0), so a structure continued in another
 * packing draws the same noise. Synchronises `stream`. */
int e3mi_md_set_langevin(e3mi_md* md, double temperature_K, double friction_per_fs, const uint64_t* seeds,
                         const int64_t* step0, void* stream);

/* Monte Carlo barostat on top of the Langevin integrator (Section 5.5: NPT
 * with a Monte Carlo barostat combined with Langevin dynamics; batched
 * systems with independent cells and seeds; Appendix D validates it). After
 * a step that brings structure s's own step count (the step0 of
 * e3mi_md_set_langevin plus the steps taken since) to a multiple of
 * `interval`, s (periodic along every axis) proposes an isotropic volume
 * change dV = (2 u0 - 1) dV_max_s, with dV_max_s = dv_max[s] (host FP64
 * [S], A^3) or, when dv_max is NULL, volume_fraction x its volume when this
 * call is made (fixed thereafter, so proposals are symmetric), scales its
 * cell lengths and positions by (V'/V)^(1/3) (velocities kept), evaluates all
 * proposals in one energy pass and accepts each with the Metropolis rule on
 *   w = E' - E + P dV - N_s kB T ln(V'/V)      (P in bar, 1 bar = 6.241509074e-7 eV/A^3)
 * i.e. accepts if w <= 0 or u1 < exp(-w / kB T); V' <= 0 is rejected.
 * u0, u1: Philox4x64-10 with key (seeds[s], 1) and counter (move_s, 0, 0, 0),
 * uniforms ((x >> 11) + 1/2) 2^-53 of the first two outputs; move_s starts at
 * move0[s] (NULL: 0) and counts proposals. seeds NULL: s. interval 0 turns
 * the barostat off. Requires e3mi_md_set_langevin with a positive friction
 * and temperature (T of the acceptance rule). Each proposal costs two
 * neighbour rebuilds and up to two energy evaluations and synchronises the
 * stream. Errors: EINVAL for open axes or bad arguments. */
int e3mi_md_set_barostat(e3mi_md* md, double pressure_bar, int interval, double volume_fraction,
                         const double* dv_max, const uint64_t* seeds, const int64_t* move0);

/* Current cells (host FP64 [S, 3, 3], rows = lattice vectors; changed by the
 * barostat) and the barostat's proposal / acceptance counts (any output may
 * be NULL). Reflects the last completed e3mi_md_step. */
int e3mi_md_cells(const e3mi_md* md, double* cells, int64_t* proposed, int64_t* accepted);

/* Total charges (host FP64 [S]) of an MD state's structures, as
 * e3mi_graph_set_total_charge; the forces of the current positions are
 * recomputed. Synchronises `stream`. */
int e3mi_md_set_total_charge(e3mi_md* md, const double* total_charge, void* stream);

/* Copy the current state to caller device buffers (any may be NULL):
 * pos, vel FP64 [N, 3], forces FP32 [N, 3]. Asynchronous on `stream`. */
int e3mi_md_state(const e3mi_md* md, double* pos, double* vel, float* forces, void* stream);

/* Counters of an MD state (any output may be NULL): steps taken, neighbour
 * rebuilds done (scheduled and early), skin violations (steps redone after an
 * early rebuild). */
int e3mi_md_stats(const e3mi_md* md, int64_t* steps, int64_t* rebuilds, int64_t* skin_violations);
int e3mi_md_destroy(e3mi_md* md);

/* Device bytes an energy_forces call needs for n_atoms atoms and n_edges skin
 * edges (graph + workspace), for admission control by a caller that packs
 * several systems. */
size_t e3mi_footprint_bytes(const e3mi_model* model, int64_t n_atoms, int64_t n_edges);

/* Per-stage timing with HIP events recorded on the launch stream, for
 * measuring kernels in place (Appendix H reports ms per MD step; this splits
 * a step into its stages). enable != 0 resets the counters and starts
 * recording; 0 stops recording and keeps the counters. Stages: prune, embed, radial_fwd, tp_fwd, mix_fwd,
 * gate_fwd, readout, gate_bwd, mix_bwd, tp_bwd_edge, radial_bwd, tp_bwd_node,
 * forces, md_update, graph_build, first_fwd, first_bwd (the species-factorised
 * first layer), last_fwd, last_bwd (the fused last layer), barostat (volume
 * moves, including their rebuilds and energy passes), coulomb (the
 * all-pairs electrostatics kernel), product_fwd, product_bwd (the product
 * block of correlation 2); "name@t" selects
 * interaction layer t.
 * e3mi_profile_query waits for the recorded events and returns the summed
 * milliseconds and the number of timed launches of a stage. */
int e3mi_profile_enable(e3mi_model* model, int enable);
int e3mi_profile_query(e3mi_model* model, const char* stage, double* total_ms, int64_t* launches);

/* Restrict the timing to one stage ("name" or "name@t"; NULL or "" for
 * every stage): only its launches are bracketed by events, so a timed run
 * can measure one kernel in place without the events of the others slowing
 * the step down (each recorded pair costs a few microseconds of device
 * time). Applies from the next launch; profile_enable keeps the selection. */
int e3mi_profile_select(e3mi_model* model, const char* stage);

/* Thread-local description of the last error ("" if none). */
const char* e3mi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* E3MI_H */
