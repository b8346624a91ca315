/*
 * mlbm.h -- C ABI of the MI355X multilevel lattice Boltzmann hot path.
 *
 * The method is the octree lattice Boltzmann scheme with the four-source
 * compact interpolation of Qi, Klimach and Roller ("Implementation of the
 * compact interpolation within the octree based Lattice Boltzmann solver
 * Musubi"): level-wise BGK pull stream-collide over sparse element arrays
 * (Sec. 2.1, Eq. bgk; Sec. 3.2), GhostFromFiner / GhostFromCoarser ghost
 * elements filled by the compact interpolation (Sec. 2.2, Eqs. compact_3D_u,
 * compact_3D_s, Steps 1-5), and acoustic time stepping in which level L+1
 * takes two steps per step of level L (Sec. 2.2).
 *
 * Conventions for every entry point:
 *   - return 0 (MLBM_OK) on success, a negative MLBM_E_* code on failure;
 *     mlbm_last_error() then describes the failure (per calling thread);
 *   - nothing is thrown across the ABI; a NULL handle gives MLBM_E_ARG;
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the device that was current at mlbm_sim_create;
 *   - all device work is enqueued on the HIP stream given to
 *     mlbm_sim_create and is asynchronous unless stated otherwise;
 *   - the library never allocates device memory: the caller provides one
 *     workspace for the simulation (and one for the adjoint) and owns it.
 *
 * Element layout (per level L, Sec. 3.2 stores fluid, then ghosts, each
 * along the space-filling curve): [fluid | GhostFromCoarser inner |
 * GhostFromCoarser outer | GhostFromFiner].  The fluid segment is itself
 * [fluid read by no interpolation | interpolation-source fluid]; every
 * part is ascending by treeID.  Per-element arrays are structure-of-arrays: component k of
 * element x is at k * n_level + x.
 */
#ifndef MLBM_H
#define MLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- enumerations --------------------------------------------------- */
enum { MLBM_D2Q9 = 0, MLBM_D3Q19 = 1, MLBM_D3Q27 = 2 };

/* Storage precision of the pdfs.  F64: double holding f_i, FP64 collision.
 * F32: float holding the deviation f_i - w_i rho0; moments and equilibria
 * in FP64, the relaxation in FP32.  F16S: half holding s_L * (f_i - w_i rho0) with a
 * power-of-two scale s_L per level; collision in FP32.  The stream-collide
 * rounds an element's diagonal directions to nearest and lets the axis pairs
 * and the rest direction absorb the accumulated momentum and mass rounding
 * errors, so each element's stored mass and momentum are off by the
 * rounding of those last values only. */
enum { MLBM_F64 = 0, MLBM_F32 = 1, MLBM_F16S = 2 };

/* Face kinds, faces ordered x-, x+, y-, y+, z-, z+.  A periodic face must
 * be paired with a periodic opposite face.  EQ supplies the equilibrium
 * f^eq(rho0, u_in) for pdfs entering through the face; COPY makes the
 * element pull its own post-collision value; WALL is halfway bounce-back.
 * When a link crosses several faces EQ wins over COPY, COPY over WALL. */
enum { MLBM_FACE_PERIODIC = 0, MLBM_FACE_EQ = 1, MLBM_FACE_COPY = 2,
       MLBM_FACE_WALL = 3 };

/* Neighbour-table codes (values < 0 in the NBR table). */
enum { MLBM_NBR_MISSING = -1, MLBM_NBR_BOUNCE = -2, MLBM_NBR_EQ = -3,
       MLBM_NBR_COPY = -4 };

/* Error codes. */
enum {
  MLBM_OK = 0,
  MLBM_E_ARG = -1,    /* bad argument, size or handle */
  MLBM_E_MESH = -2,   /* invalid mesh: tiling, 2:1 jumps, ghost sources */
  MLBM_E_STATE = -3,  /* call out of order (e.g. step before init) */
  MLBM_E_HIP = -4,    /* a HIP runtime call failed */
  MLBM_E_OOM = -5     /* host allocation failed */
};

/* Diagnostics mask bits and status flags. */
enum { MLBM_DIAG_MASS = 1, MLBM_DIAG_KE = 2, MLBM_DIAG_FORCE = 4 };
/* MLBM_STATUS_GRAPH_FALLBACK: recording or instantiating the HIP graph of
 * mlbm_step failed, and the simulation launches its kernels directly from
 * then on (same results, more launch overhead) until mlbm_use_graphs(1). */
enum { MLBM_STATUS_NONFINITE = 1, MLBM_STATUS_F16_OVERFLOW = 2,
       MLBM_STATUS_GRAPH_FALLBACK = 4 };

/* Exportable plan tables (mlbm_plan_export). */
enum {
  MLBM_TABLE_TREEID = 0,   /* uint64 [n]: treeIDs in layout order          */
  MLBM_TABLE_COORDS = 1,   /* int32 [d][n]: integer coords on the level     */
  MLBM_TABLE_NBR = 2,      /* int32 [q-1][n]: pull source of direction i>=1 */
  MLBM_TABLE_GFC_SRC = 3,  /* int32 [4][n_gfc]: H,K,M,N (3D) or P,Px,Py,Pxy
                              (2D) element indices on level L-1             */
  MLBM_TABLE_GFF_SRC = 4,  /* int32 [4][n_gff]: source element indices on
                              level L+1                                      */
  MLBM_TABLE_CAPTURE = 5,  /* int32 [n_cap_fluid]: fluid elements whose
                              pre-collision moments are captured (the tail
                              of the fluid segment)                         */
  MLBM_TABLE_BOUNCE = 6,   /* int32 [2][n_bounce]: (element, direction i)
                              fluid links whose pull source is solid        */
  /* The NBR table over the updated elements as the device holds it, in
   * blocks of 256 elements, with H = NBR_HDR[b] = {regmask, kself, w, 0}.
   * Direction i >= 1 of block b is "Morton" if bit i of regmask is set:
   * with m = x + kself and mo = the Morton code of x - c_i formed from m by
   * dilated arithmetic, all mod 2^32 (the level-local Morton code is the
   * treeID minus the level's first treeID), and {k0, k1, t0, t1} =
   * NBASE[b][i-1], the source is mo + ((mo - t0) >= t1 ? k1 : k0)
   * (unsigned compare); its codes are not read.  Otherwise code c of
   * element x: c >= 0xFFFC is the link code c - 0x10000 (-4..-1), else the
   * source is NBASE[b][i-1][c >> 14] + (c & 0x3FFF).  A block with w >= 0
   * is wide (regmask 0): its entry is the int32
   * (NBR_WIDE[i-1][w * 256 + x - 256 b] << 16) | c. */
  MLBM_TABLE_NBR16 = 7,    /* uint16 [q-1][n_blocks * 256]                  */
  MLBM_TABLE_NBASE = 8,    /* int32 [n_blocks][q-1][4]                      */
  MLBM_TABLE_NBR_WIDE = 9, /* uint16 [q-1][n_wide * 256]                    */
  MLBM_TABLE_NBR_HDR = 10, /* int32 [n_blocks][4]                           */
  /* Links that carry a wall fraction (mlbm_plan_set_walls), sorted by
   * element then direction: {element x, pull direction j (its source
   * x - c_j is solid), second node x2 = the element at x + c_j (the pull
   * source of opp(j); -1 if that is not an element), weight class}. */
  MLBM_TABLE_WALL = 11,    /* int32 [n_wall][4]                             */
  MLBM_TABLE_WALL_Q = 12   /* double [n_wall]: wall fraction q of each link */
};

/* Fields of mlbm_plan_level_info, in this order (int64 each). */
enum {
  MLBM_INFO_LEVEL = 0, MLBM_INFO_N = 1, MLBM_INFO_N_FLUID = 2,
  MLBM_INFO_N_GFC_INNER = 3, MLBM_INFO_N_GFC_OUTER = 4, MLBM_INFO_N_GFF = 5,
  MLBM_INFO_N_CAP_FLUID = 6, MLBM_INFO_N_CAP = 7, MLBM_INFO_N_GFC_GROUPS = 8,
  MLBM_INFO_N_BOUNCE = 9, MLBM_INFO_N_WALL = 10, MLBM_INFO_FIELDS = 11
};

/* State selectors for mlbm_get_state / mlbm_set_state.  The stored state of
 * a level is post-collision (pull scheme); the pre-collision pdfs of the
 * fluid elements at the same time are those its last stream-collide
 * gathered (Sec. 2.1: the strain rate is a moment of these).  A level keeps
 * the array that stream-collide read, so they are formed again on request
 * by the same pull; selectors marked (*) need a stream-collide of the level
 * since its state was last set by mlbm_init, mlbm_set_state or
 * mlbm_load_checkpoint (else MLBM_E_STATE). */
enum {
  MLBM_STATE_PDF_POST = 0, /* post-collision pdfs f*, all elements, FP64
                              [q][n]                                          */
  MLBM_STATE_MOMENTS = 1,  /* rho, u of fluid elements, FP64 [1+d][n_fluid] */
  MLBM_STATE_PDF_PRE = 2,  /* (*) pre-collision pdfs f of the fluid
                              elements, FP64 [q][n_fluid]                     */
  MLBM_STATE_STRAIN = 3,   /* (*) strain rate of the fluid elements from those
                              pdfs (Sec. 2.1), S_ab = -(3 omega_L/(2 rho))
                              sum_i c_ia c_ib f^neq_i, f^neq = f - f^eq(rho,u),
                              level-L lattice units, FP64 [d(d+1)/2][n_fluid]
                              in the order xx, yy, zz, xy, yz, xz (2D: xx, yy,
                              xy); no division by 1 - omega, so tau = 1 is
                              fine                                            */
  MLBM_STATE_PDF_PREV = 4  /* (*) the post-collision state the last
                              stream-collide read (one level substep earlier,
                              wall-link values included), all elements, FP64
                              [q][n]; ghosts that stream-collide did not read
                              hold older values                               */
};

typedef struct mlbm_plan mlbm_plan;
typedef struct mlbm_sim mlbm_sim;

/* ---- errors --------------------------------------------------------- */
/* Human-readable name of an error code (static string). */
const char* mlbm_error_string(int32_t code);
/* Message of the last failure on the calling thread ("" if none). */
const char* mlbm_last_error(void);

/* ---- lattice -------------------------------------------------------- */
/* Velocity set used by the library for `stencil` (Sec. 2.1): writes q,
 * then c (int32 [q][d], host) and w (double [q], host) if non-NULL.
 * Direction 0 is the rest velocity.  Host only. */
int32_t mlbm_lattice(int32_t stencil, int32_t* q, int32_t* c, double* w);

/* ---- plan: host-only mesh analysis (Sec. 3.1, 3.2; Sec. 2.2 ghosts) --- */
/* Build all level-wise tables from the leaf treeIDs of the fluid elements
 * (any order) and the treeIDs of solid cells.  treeID numbering: root id 0
 * at level 0, children of t are 2^d t + 1 ... 2^d t + 2^d with the Morton
 * bit order x, y, z.  box_origin / box_extent (d entries each) give the
 * domain in cells of level `level0`, the coarsest level present.  face_bc
 * has 2d entries.  Host arrays are copied; the plan owns its memory until
 * mlbm_plan_destroy.  Errors: MLBM_E_ARG (bad sizes/enums), MLBM_E_MESH
 * (elements outside the box, holes or overlaps, a ghost source that is not
 * fluid / GhostFromFiner, or an updated element missing a neighbour).
 * Needs no GPU. */
int32_t mlbm_plan_create(int32_t stencil, int32_t level0,
                         const int32_t* box_origin, const int32_t* box_extent,
                         const int32_t* face_bc,
                         const uint64_t* leaf_ids, int64_t n_leaves,
                         const uint64_t* solid_ids, int64_t n_solids,
                         mlbm_plan** out);
void mlbm_plan_destroy(mlbm_plan* plan);
/* Policy for Morton directions of the device pull table (MLBM_TABLE_NBR_HDR)
 * in plans created after the call: a block uses them if at least
 * block_min_directions of its directions qualify (1..26), a level if they
 * cover at least level_min_fraction (0..1) of its (block, direction) pairs;
 * defaults 0 and 6.  Results do not depend on it, only the traffic and
 * instruction mix of the stream-collide.  Process-wide; not to be called
 * while another thread creates a plan.  MLBM_E_ARG for values out of range. */
int32_t mlbm_set_morton_policy(double level_min_fraction, int32_t block_min_directions);
/* Curved walls (Sec. 2.3; linear interpolated bounce-back of Bouzidi,
 * Firdaouss and Lallemand): link t runs from the fluid leaf ids[t] along
 * lattice velocity dirs[t] (mlbm_lattice order, pointing into the solid)
 * to a solid cell; the wall cuts it at fraction q[t] in [0, 1] of the link
 * from the element's centre.  With i = dirs[t], ibar = opp(i) and x2 the
 * element at x - c_i, the stream step then takes
 *   q <  1/2: f_ibar(x, t+1) = 2q f*_i(x) + (1 - 2q) f*_i(x2)
 *             (halfway bounce-back f*_i(x) where x - c_i is no element)
 *   q >= 1/2: f_ibar(x, t+1) = f*_i(x)/(2q) + (1 - 1/(2q)) f*_ibar(x)
 * instead of halfway bounce-back, and the momentum-exchange force
 * (MLBM_DIAG_FORCE) sums c_i (f*_i(x) + f_ibar(x, t+1)) over its links.
 * Replaces the plan's previous set (n = 0 clears it).  Host arrays are
 * copied.  Affects simulations created afterwards, whose workspace grows
 * (query mlbm_sim_workspace_bytes after this call).  The adjoint covers
 * the links (the transposed rule and the drag seed of the interpolated
 * values); its workspace grows with them.  Errors (the plan is left
 * unchanged): MLBM_E_ARG (NULL arrays with n > 0, a direction out of
 * range, q outside [0, 1] or not finite, a link given twice), MLBM_E_MESH
 * (an id that is not a fluid leaf, or a link whose neighbour is not
 * solid).  Host only. */
int32_t mlbm_plan_set_walls(mlbm_plan* plan, const uint64_t* ids, const int32_t* dirs,
                            const double* q, int64_t n);
/* GhostFromCoarser layers of plans created after the call (Sec. 2.2, last
 * paragraph): 2 (default) for acoustic scaling, two fine steps per coarse
 * step; 4 for diffusive scaling, four fine steps per coarse step.  Distances
 * 1 .. layers-1 from fine fluid form the inner part (MLBM_INFO_N_GFC_INNER),
 * distance `layers` the outer layer.  A simulation of a 4-layer plan runs
 * the diffusive schedule (see mlbm_sim_create, mlbm_step); its adjoint and
 * its force are not available (MLBM_E_STATE).  Process-wide; not to be
 * called while another thread creates a plan.  MLBM_E_ARG for other
 * values. */
int32_t mlbm_set_gfc_layers(int32_t layers);
/* The GhostFromCoarser layer count the plan was built with. */
int32_t mlbm_plan_gfc_layers(const mlbm_plan* plan, int32_t* layers);
/* Number of levels (Lmax - L0 + 1) and L0. */
int32_t mlbm_plan_levels(const mlbm_plan* plan, int32_t* n_levels,
                         int32_t* level0);
/* MLBM_INFO_FIELDS int64 values describing level index k (0 = coarsest). */
int32_t mlbm_plan_level_info(const mlbm_plan* plan, int32_t k, int64_t* out);
/* Copy table `table` of level index k into host memory; `bytes` must equal
 * the table's size exactly (query it with dst = NULL, which stores the
 * size in *bytes). */
int32_t mlbm_plan_export(const mlbm_plan* plan, int32_t k, int32_t table,
                         void* host_dst, size_t* bytes);

/* ---- simulation ------------------------------------------------------ */
/* Device workspace bytes a simulation of `plan` at `precision` needs. */
int32_t mlbm_sim_workspace_bytes(const mlbm_plan* plan, int32_t precision,
                                 size_t* bytes);
/* Create a simulation bound to `hip_stream` (a hipStream_t, may be NULL for
 * the null stream) using the caller's device `workspace` (256-byte aligned,
 * at least mlbm_sim_workspace_bytes).  tau0 is the BGK relaxation time of
 * level L0; finer levels follow Eq. fneq_scale with m = 2 (acoustic
 * scaling), or all levels take tau0 for a plan with four GhostFromCoarser
 * layers (diffusive scaling: dx halves and dt quarters per level, so
 * nu dt / dx^2 is level invariant).  rho0 is the
 * reference density (shift of F16S storage and density of EQ faces),
 * u_in (d doubles, host, may be NULL = 0) the EQ-face velocity.  f16_exp
 * (n_levels ints, host) sets s_L = 2^f16_exp[k] for F16S; NULL picks it at
 * mlbm_init from the initial state.  Uploads the index tables (enqueued on
 * the stream).  The workspace must outlive the simulation. */
int32_t mlbm_sim_create(const mlbm_plan* plan, int32_t precision, double tau0,
                        double rho0, const double* u_in, const int32_t* f16_exp,
                        void* hip_stream, void* workspace,
                        size_t workspace_bytes, mlbm_sim** out);
void mlbm_sim_destroy(mlbm_sim* sim);

/* Initial state of level index k (Sec. 4.1 initialisation): for every fluid
 * element f = f^eq(rho, u) + f^neq(S), f^neq_i = -(w_i rho/(cs^2 omega_L))
 * Q_i:S.  Device FP64 arrays over the level's fluid elements in layout
 * order: rho [n_fluid], u [d][n_fluid], S [d(d+1)/2][n_fluid] with
 * components xx, yy, zz, xy, yz, xz (2D: xx, yy, xy) in level-L lattice
 * units; S may be NULL (zero).  Call for every level, then
 * mlbm_fill_ghosts. */
int32_t mlbm_init(mlbm_sim* sim, int32_t k, const double* rho, const double* u,
                  const double* S);
/* Synchronous ghost fill (Sec. 2.2): all GhostFromFiner, then all
 * GhostFromCoarser, from the pre-collision moments captured at the last
 * synchronous time. */
int32_t mlbm_fill_ghosts(mlbm_sim* sim);
/* Advance n coarse steps with the recursive schedule: advance(L) = one
 * stream-collide of L; if L < Lmax: advance(L+1) twice (four times under
 * diffusive scaling), fill GhostFromFiner(L), fill GhostFromCoarser(L+1).
 * Under diffusive scaling the fills also take velocity and density
 * deviation between the levels' lattice units (factor 2 and 4 per level,
 * fine to coarse).  Asynchronous.  Pairs of
 * coarse steps are replayed from an instantiated HIP graph (recorded once
 * per parity state on an internal stream, launched on the bound stream);
 * the results are identical to direct launches. */
int32_t mlbm_step(mlbm_sim* sim, int64_t n_coarse);
/* Enable (default) or disable graph replay in mlbm_step. */
int32_t mlbm_use_graphs(mlbm_sim* sim, int32_t enable);
/* FP64 reductions written to device memory `dev_out` (deterministic, no
 * atomics): for each bit set in `mask` in the order MASS (1 value),
 * KE (1), FORCE (d).  MASS = sum_L V_L sum_fluid rho; KE = 1/2 sum_L V_L
 * sum_fluid rho |u|^2 with V_L = 2^(-d (L - L0)), density deviation and
 * velocity in level-L0 lattice units (under diffusive scaling a level-L
 * value is taken to L0 units by 2^(L-L0), squared for the density
 * deviation); FORCE = momentum exchange (Sec. 2.3) over bounce-back links,
 * each level scaled to finest-level units by 2^((d-1)(Lmax - L)), acoustic
 * scaling only (MLBM_E_STATE otherwise). */
int32_t mlbm_diagnostics(mlbm_sim* sim, uint32_t mask, double* dev_out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * reductions of mlbm_diagnostics, bit for bit, with the per-block partials
 * in a static scratch array of the library (one per GPU, 320 KiB, held
 * until the process ends) instead of the simulation's workspace.  At most
 * 16 levels (MLBM_E_ARG otherwise).  All calls on one GPU share that array:
 * calls that overlap on a GPU (different streams, or simulations on other
 * host threads) race and give undefined results; calls ordered on one
 * stream do not.  Allocates nothing. */
int32_t mlbm_diagnostics_noalloc(mlbm_sim* sim, uint32_t mask, double* dev_out);
/* Copy state `what` (MLBM_STATE_*) of level index k to device memory
 * `dev_dst`, laid out as the selector states (the caller allocates it).
 * Errors: MLBM_E_ARG (unknown selector, level out of range, NULL),
 * MLBM_E_STATE (the level has no state yet; a (*) selector before the
 * level's first stream-collide since its state was set). */
int32_t mlbm_get_state(mlbm_sim* sim, int32_t k, int32_t what, double* dev_dst);
/* Set the state of level index k from device FP64 memory `dev_src`.
 * what = MLBM_STATE_PDF_POST: [q][n], the post-collision pdfs of all
 * elements are overwritten (test states; capture records are left as they
 * are).  what = MLBM_STATE_PDF_PRE: [q][n_fluid], pre-collision pdfs of the
 * fluid elements: they are collided with the level's omega (Eq. bgk) and
 * stored, and the interpolation sources among them record their moments,
 * as a stream-collide does after its gather; mlbm_fill_ghosts then fills
 * the ghosts from them (Sec. 2.2, Steps 1-5).  Ghost entries are left
 * unchanged.  Other selectors: MLBM_E_ARG. */
int32_t mlbm_set_state(mlbm_sim* sim, int32_t k, int32_t what, const double* dev_src);
/* Sticky device status flags (MLBM_STATUS_*); synchronises the stream.
 * The flags are cleared after reading. */
int32_t mlbm_status(mlbm_sim* sim, uint32_t* flags);
/* Number of coarse steps taken since mlbm_init. */
int32_t mlbm_time(const mlbm_sim* sim, int64_t* coarse_steps);

/* Checkpoint: raw per-level pdf arrays, capture buffers, parities and the
 * step counter.  Device-to-device copies on the stream; `bytes` must be at
 * least mlbm_checkpoint_bytes.  A run restored by load_checkpoint continues
 * bit-identically. */
int32_t mlbm_checkpoint_bytes(const mlbm_sim* sim, size_t* bytes);
int32_t mlbm_save_checkpoint(mlbm_sim* sim, void* dev_dst, size_t bytes);
int32_t mlbm_load_checkpoint(mlbm_sim* sim, const void* dev_src, size_t bytes);

/* The number of kernel launches one coarse step enqueues. */
int32_t mlbm_launches_per_step(const mlbm_sim* sim, int64_t* launches);

/* Kernel timing.  While enabled, every stream-collide launch is bracketed
 * by HIP events recorded on the bound stream; enabling synchronises the
 * stream and clears earlier records.  mlbm_profile_read (synchronises)
 * returns, for level index k, the summed bracketed time in milliseconds,
 * the number of launches and the summed number of elements updated. */
int32_t mlbm_profile(mlbm_sim* sim, int32_t enable);
int32_t mlbm_profile_read(mlbm_sim* sim, int32_t k, double* ms, int64_t* launches,
                          int64_t* elements);
/* As mlbm_profile_read for kernel kind 0 (forward stream-collide) or 1
 * (adjoint stream-collide, bracketed inside mlbm_adjoint_step). */
int32_t mlbm_profile_read_kind(mlbm_sim* sim, int32_t kind, int32_t k, double* ms,
                               int64_t* launches, int64_t* elements);

/* ---- adjoint ----------------------------------------------------------
 * Hand-written reverse of the multilevel step (adjoints of Eq. bgk, of the
 * pull streaming and of both compact-interpolation fills, Steps 1-5), for
 * gradients of an objective of the final state with respect to the
 * initial fields, tau0 and the EQ-face velocity.  lambda arrays hold
 * dJ/d(f*) per level in the simulation's compute precision; the FP16
 * storage rounding is treated as the identity.  Usage: attach a workspace;
 * run the forward to time T; seed; call mlbm_adjoint_step with the
 * checkpoint of the start of each coarse step, last step first; finish
 * with mlbm_adjoint_init; read the parameter gradients. */
enum { MLBM_OBJ_KE = 0, MLBM_OBJ_DRAG_X = 1 };

/* Device workspace bytes for the adjoint of `sim`, which was created from
 * `plan` (the plan must still exist; its transposed tables are used). */
int32_t mlbm_adjoint_workspace_bytes(const mlbm_sim* sim, const mlbm_plan* plan,
                                     size_t* bytes);
/* Attach a caller-owned, 256-byte aligned device workspace (the tape of one
 * coarse step, lambda arrays and transposed tables).  Synchronises. */
int32_t mlbm_adjoint_attach(mlbm_sim* sim, const mlbm_plan* plan, void* workspace,
                            size_t bytes);
/* lambda := dJ/df* of the simulation's current state for objective
 * MLBM_OBJ_KE (kinetic energy, as MLBM_DIAG_KE) or MLBM_OBJ_DRAG_X (x force,
 * as MLBM_DIAG_FORCE); clears the parameter accumulators. */
int32_t mlbm_adjoint_seed(mlbm_sim* sim, int32_t objective);
/* Reverse one coarse step.  `dev_ckpt` (device, `bytes` >= checkpoint size)
 * is the mlbm_save_checkpoint image of the state at the START of the coarse
 * step whose end-state adjoint lambda holds; afterwards lambda refers to
 * that start state.  The step's kernels read the checkpoint in place: keep
 * it unchanged until the bound stream has passed this step.  The
 * simulation's own arrays are not modified. */
int32_t mlbm_adjoint_step(mlbm_sim* sim, const void* dev_ckpt, size_t bytes);
/* Reverse the initialisation and the initial synchronous fill.  rho, u, S
 * are host arrays of n_levels device pointers to the inputs given to
 * mlbm_init (S may be NULL or hold NULL entries); dJ_du (required) and
 * dJ_drho, dJ_dS (optional, NULL) are host arrays of n_levels device
 * pointers receiving FP64 gradients laid out like the inputs. */
int32_t mlbm_adjoint_init(mlbm_sim* sim, const double* const* rho,
                          const double* const* u, const double* const* S,
                          double* const* dJ_du, double* const* dJ_drho,
                          double* const* dJ_dS);
/* Accumulated parameter gradients (synchronises): dJ/dtau0 through all
 * levels' omega_L (Eq. fneq_scale), dJ/domega_L per level (n_levels
 * doubles, may be NULL) and dJ/du_in (3 doubles, may be NULL). */
int32_t mlbm_adjoint_params(mlbm_sim* sim, double* dJ_dtau0, double* dJ_domega,
                            double* dJ_duin);
/* Copy lambda of level index k to device FP64 [q][n]. */
int32_t mlbm_adjoint_get_lambda(mlbm_sim* sim, int32_t k, double* dev_dst);

#ifdef __cplusplus
}
#endif
#endif /* MLBM_H */
