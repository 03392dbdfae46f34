/*
 * plbm.h -- C ABI of libplbm, the MI355X (gfx950) implementation of the
 * pseudo-potential lattice Boltzmann (P-LBM) update of Czelusniak, Bingert,
 * Krause and Simonis, "On the consistency of pseudo-potential lattice
 * Boltzmann methods" (arXiv 2504.15018).
 *
 * What one step computes (Sec. II of the paper, lattice units dx = dt = 1,
 * G = -1):
 *   rho = sum_i f_i                                   eq. (Density)
 *   psi = sqrt(2 (rho/3 - p_EOS(rho)))                eq. (Interaction_Potential)
 *   M1, M2 = stencil moments of psi over all directions  (Sec. II, M^(1), M^(2))
 *   F   = -G psi M1 + (G/4) eps M1.M2 - (G/6)(kappa-1)(M1.M2 - M1 tr M2) + F_g
 *                                                     eq. (interactionForce);
 *         the eps coefficient is the one that reproduces the paper's pressure
 *         tensor, eq. (New_Pressure_Tensor)
 *   u   = (sum_i f_i c_i + F/2) / rho                 eq. (Momentum)
 *   tau = tau_v + (rho - rho_v)/(rho_l - rho_v) (tau_l - tau_v)   (Sec. VI)
 *   BGK collision, eq. (LBE), with Guo forcing, eq. (Guo_Forcing_Scheme), or
 *   the MRT extension; streaming with periodic wrap or half-way bounce-back.
 *
 * Conventions for every call:
 *   - Every function returns an int status: PLBM_OK (0) or a negative
 *     PLBM_E_* code.  No C++ exception crosses this boundary.  On error,
 *     plbm_last_error() returns a message (thread-local, owned by the library,
 *     valid until the next call on the same thread).
 *   - Populations and fields exchanged with the caller are float64, in
 *     structure-of-arrays layout with x fastest: f[q][z][y][x] (3-D) or
 *     f[q][y][x] (2-D); vector fields u[a][...] likewise, a = 0..d-1.
 *   - D2Q9 direction order is that of eq. (VelocitySet): rest, (1,0), (0,1),
 *     (-1,0), (0,-1), (1,1), (-1,1), (-1,-1), (1,-1).
 *     D3Q19 order: rest; (1,0,0), (-1,0,0), (0,1,0), (0,-1,0), (0,0,1),
 *     (0,0,-1); (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1),
 *     (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).
 *   - Device memory is owned by the caller (for example a PyTorch uint8
 *     tensor); the library never allocates device memory.  Host buffers
 *     passed in are read or written during the call only.
 *   - Handles are not thread-safe; use one handle per stream.
 */
#ifndef PLBM_H
#define PLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PLBM_ABI_VERSION 4

/* status codes */
#define PLBM_OK 0
#define PLBM_E_INVALID (-1)     /* argument out of range or inconsistent */
#define PLBM_E_UNSUPPORTED (-2) /* combination not built (see plbm_create) */
#define PLBM_E_NOMEM (-3)       /* caller's device buffer too small */
#define PLBM_E_DEVICE (-4)      /* HIP runtime error; message carries the HIP string */
#define PLBM_E_UNSTABLE (-5)    /* health flags raised (NaN, rho <= 0) */
#define PLBM_E_NOCONVERGE (-6)  /* parameter root solve did not converge */

/* lattice kinds */
#define PLBM_D2Q9 0
#define PLBM_D3Q19 1
/* collision operators */
#define PLBM_BGK 0
#define PLBM_MRT 1
/* population storage */
#define PLBM_F64 0   /* float64 storage and arithmetic */
#define PLBM_F32 1   /* float32 storage and arithmetic; psi(rho) evaluated in float64 */
#define PLBM_F16S 2  /* IEEE half storing f_i - w_i rho0; float32 arithmetic; float64 psi */
#define PLBM_BF16S 3 /* bfloat16 storing f_i - w_i rho0; float32 arithmetic; float64 psi */
/* Locally shifted 16-bit storage: f_i - w_i rho_ref(x), with rho_ref(x) a
 * per-node reference density (the node's density at the previous step,
 * rounded to half precision, kept in an extra 2-byte-per-node A-B array and
 * counted by plbm_lattice_bytes).  Every population is encoded with the
 * reference of the node that decodes it, so the reference's own rounding
 * costs nothing; the stored deviation is the non-equilibrium and velocity
 * part only, which keeps vapour and liquid at the same relative precision.
 * Extra traffic: 4 bytes per node update.  float32 arithmetic, float64 psi. */
#define PLBM_F16R 4
#define PLBM_BF16R 5
/* population storage patterns */
#define PLBM_PATTERN_AB 0 /* two population arrays; one fused kernel per step (2 Q S bytes per node) */
/* In-place (AA) pattern: one population array.  Even steps read and write
 * a node's own Q slots (writing each post-collision population into the
 * opposite direction's slot); odd steps read from and write to the
 * neighbours' slots, so each node touches only slots no other node touches
 * and the update is in place.  The neighbours' psi cannot be read from
 * populations that may already be overwritten, so each step is a psi pass
 * (Q S read, one psi value written per node) and the update (2 Q S plus the
 * psi stencil): about 1.5x the traffic of the A-B pattern for half its
 * population memory.  Results equal those of the A-B pattern, in every
 * storage format (with locally shifted storage the psi pass also writes the
 * nodes' new reference densities). */
#define PLBM_PATTERN_AA 1
/* discretisations of the two-phase force */
#define PLBM_SCHEME_PSEUDOPOTENTIAL 0 /* the paper's update: psi stencil force, eq. (interactionForce) */
/* Well-balanced discretisation (the class of schemes Sec. VI.B names as the
 * cure for spurious currents; the paper gives no equations, so this is the
 * library's reading): the force is written in potential form
 * F = -rho grad_d mu + F_g with the lattice chemical potential
 * mu = mu_b(rho) - k lap_d rho (mu_b: the bulk chemical potential of the same
 * EOS, d mu_b/d rho = p'(rho)/rho; k: gradient coefficient wb_k; grad_d and
 * lap_d the isotropic lattice stencils), and the equilibrium carries the
 * constant wb_rho0 on the moving populations at rest
 * (f_i^eq = w_i wb_rho0 + delta_i0 (rho - wb_rho0) + w_i rho s_i(u)).  A fluid
 * at rest with uniform mu is then an exact steady state: spurious currents
 * decay to round-off.  Coexistence follows Maxwell's construction; the
 * surface tension is int k rho'^2 dx; epsilon and kappa are not used.
 * Per step: a chemical-potential pass (densities of the pulled populations,
 * mu of every node into one extra value per node, counted by
 * plbm_lattice_bytes), then the update.  Supported with the A-B pattern, F64
 * or F32 storage, mirror walls, alone or in a batch. */
#define PLBM_SCHEME_WELL_BALANCED 1
/* boundary kinds, per axis */
#define PLBM_PERIODIC 0
#define PLBM_HALFWAY_BB 1 /* walls half a spacing outside the first and last node */
/* equations of state */
#define PLBM_EOS_PAPER 0        /* eq. (EOS) of Sec. IV */
#define PLBM_EOS_PENG_ROBINSON 1 /* Peng-Robinson, lattice constants a = 2/49, b = 2/21, R = 1 */
/* health flags of plbm_diag.flags */
#define PLBM_FLAG_NAN 1
#define PLBM_FLAG_RHO_NONPOS 2
#define PLBM_FLAG_PSI_NEG 4 /* psi radicand < 0 somewhere (clamped to 0) */

/* Physical (SI) description of the fluid and problem (Sec. V, Table I). */
typedef struct plbm_phys_params {
  int32_t eos;           /* PLBM_EOS_* */
  int32_t pad0;
  double rho_v, rho_l;   /* kg/m^3: coexistence densities (paper EOS: imposed) */
  double nu_v, nu_l;     /* m^2/s: kinematic viscosities of vapour and liquid */
  double gamma;          /* N/m: surface tension; <= 0 selects kappa = 1 */
  double xi;             /* m: interface width (paper EOS, eq. thickness) */
  double L;              /* m: characteristic length L_phs of eq. (unit) */
  double body_force[3];  /* N/m^3 */
  double T_over_Tc;      /* Peng-Robinson: reduced temperature */
  double omega;          /* Peng-Robinson: acentric factor */
  double epsilon;        /* mechanical-stability parameter; 0 selects 2 (Sec. IV) */
  double U_phys;         /* m/s: optional characteristic velocity for Re (0: none) */
} plbm_phys_params;

/* The converter's three lattice inputs, eq. (unit): L_lat, nu_l,lat (through
 * tau_l, nu = (tau - 1/2)/3), rho_l,lat. */
typedef struct plbm_lattice_map {
  double L_lat;
  double tau_l;
  double rho_l_lat; /* 0 selects 1.187 (Sec. VI) */
} plbm_lattice_map;

/* Resolved constants in lattice units, as consumed by plbm_create. */
typedef struct plbm_lattice_params {
  int32_t eos;
  int32_t pad0;
  double K;                    /* paper EOS: p_c / rho_c^3 from eq. (thickness) */
  double eos_rho_v, eos_rho_l; /* paper EOS: the densities inside eq. (EOS) */
  double pr_a, pr_b, pr_R, pr_T, pr_alpha; /* Peng-Robinson constants */
  double rho_v, rho_l;         /* coexistence densities predicted by the
                                  mechanical-stability condition (Sec. IV);
                                  they anchor tau(rho) */
  double epsilon, kappa, G;    /* eq. (interactionForce); G = -1 */
  double tau_v, tau_l;         /* relaxation times of vapour and liquid */
  double body_force[3];        /* lattice units */
  double C_L, C_T, C_M, C_U, C_VF, C_gamma, C_p; /* eqs. (unit), (unit2); 0 if none */
  double Re;                   /* U_phys L / nu_l when U_phys > 0, else 0 */
  double gamma_lat;            /* lattice surface tension (0 if kappa set directly) */
} plbm_lattice_params;

/* Geometry, operator and storage of one lattice. */
typedef struct plbm_lattice_desc {
  int32_t lattice;   /* PLBM_D2Q9 | PLBM_D3Q19 */
  int32_t collision; /* PLBM_BGK | PLBM_MRT */
  int32_t storage;   /* PLBM_F64 | PLBM_F32 | PLBM_F16S | PLBM_BF16S | PLBM_F16R | PLBM_BF16R */
  int32_t nx, ny, nz; /* nodes per axis; D2Q9 uses nx, ny and requires nz = 1 */
  int32_t bc[3];      /* per axis x, y, z: PLBM_PERIODIC or PLBM_HALFWAY_BB.
                         Walls are supported on the last axis only (z in 3-D,
                         y in 2-D); other axes must be periodic. */
  int32_t pattern;    /* PLBM_PATTERN_AB | PLBM_PATTERN_AA */
  double rho0_shift;  /* reference density of shifted storage (F16S/BF16S);
                         0 selects rho_l of the parameters */
  double mrt_rates[4]; /* MRT rates s_e, s_eps, s_q, s_m; 0 selects 0.8, 0.8,
                          1.1, 1.1.  Stress (and D3Q19 pi) moments relax at
                          1/tau(rho); momentum moments are rate-independent. */
  double rho_wall[2];  /* wetting walls (an extension beyond the paper's solid
                          walls): the psi ghost beyond the wall below / above
                          is psi(rho_wall) instead of the mirror of the
                          wall-adjacent node, which sets the contact angle
                          (rho_wall near rho_l wets, near rho_v does not).
                          0 keeps the neutral mirror ghost.  Requires walls;
                          must be finite and >= 0. */
  int32_t scheme;      /* PLBM_SCHEME_PSEUDOPOTENTIAL (0) | PLBM_SCHEME_WELL_BALANCED */
  int32_t pad1;
  double wb_k;         /* well-balanced scheme: gradient coefficient k > 0 */
  double wb_rho0;      /* well-balanced scheme: reference density of the moving
                          equilibrium populations; 0 selects rho_v of the
                          parameters */
} plbm_lattice_desc;

/* Initial density shape evaluated on the device (tanh interfaces of width W,
 * nodes at integer positions). */
#define PLBM_SHAPE_SLAB 0    /* liquid in the central half of axis `axis` */
#define PLBM_SHAPE_DROPLET 1 /* liquid sphere/disc of radius R at centre[] */
#define PLBM_SHAPE_LAYERS 2  /* liquid below `level` along axis `axis` */
typedef struct plbm_shape {
  int32_t kind;
  int32_t axis;
  double rho_in, rho_out; /* liquid and vapour densities */
  double W;               /* interface width parameter */
  double R;               /* droplet radius */
  double centre[3];       /* droplet centre */
  double level;           /* layer height */
  double u0[3];           /* uniform initial velocity */
} plbm_shape;

/* Global diagnostics of one lattice at its current time. */
typedef struct plbm_diag {
  double mass;            /* sum rho, compensated float64 sum */
  double mass_comp_err;   /* magnitude of the compensation term */
  double momentum[3];     /* sum rho u (u includes F/2, eq. Momentum) */
  double max_u;           /* max |u| */
  double max_du_per_step; /* max |u(t) - u(t_prev)| / (t - t_prev) since the previous
                             plbm_reduce on this lattice (0 on the first call) */
  int64_t time;           /* steps taken */
  int32_t flags;          /* PLBM_FLAG_* */
  int32_t pad0;
} plbm_diag;

typedef struct plbm_lattice plbm_lattice;
typedef struct plbm_batch plbm_batch;

/* ABI version of the loaded library (PLBM_ABI_VERSION). */
int plbm_abi_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* plbm_last_error(void);

/* Unit conversion and parameter derivation (host only, float64).
 * eqs. (unit), (unit2): conversion factors from L_phs/L_lat, tau_l and
 * rho_l,lat; eq. (thickness): K = p_c/rho_c^3 from the interface width xi;
 * eq. (surface_tension): kappa from gamma (f_gamma with rho_v, rho_l as in
 * Appendix B); tau_v from nu_v; body force / C_VF.  For Peng-Robinson the
 * lattice EOS is fixed by T_over_Tc and omega, and rho_v, rho_l are solved
 * from the mechanical-stability condition.
 * Errors: PLBM_E_INVALID (rho_v >= rho_l, tau_l <= 1/2, xi <= 0, L <= 0, ...),
 * PLBM_E_NOCONVERGE (root solve). */
int plbm_resolve_params(const plbm_phys_params* phys, const plbm_lattice_map* map, plbm_lattice_params* out);

/* Lattice-unit Peng-Robinson parameters (Yuan-Schaefer constants) at
 * T/Tc and acentric factor omega; rho_v, rho_l from the mechanical-stability
 * condition of Sec. IV at this epsilon.  body_force may be NULL. */
int plbm_params_pr_lattice(double T_over_Tc, double omega, double epsilon, double kappa, double tau_v,
                           double tau_l, const double* body_force, plbm_lattice_params* out);

/* Lattice-unit paper-EOS parameters: eq. (EOS) with coexistence rho_v, rho_l
 * and K from the width xi (eq. thickness); rho_v/rho_l of the output are the
 * finite-psi mechanical-stability prediction at this epsilon.
 * body_force may be NULL. */
int plbm_params_paper_lattice(double rho_v, double rho_l, double xi, double epsilon, double kappa,
                              double tau_v, double tau_l, const double* body_force, plbm_lattice_params* out);

/* Exact device bytes plbm_create needs for this descriptor: two population
 * arrays (A-B pattern), float64 staging for moments/fields, the previous
 * velocity for the convergence residual, reduction partials. */
int plbm_lattice_bytes(const plbm_lattice_desc* desc, uint64_t* bytes);

/* Bind a lattice to caller-owned device memory dev_mem (at least
 * plbm_lattice_bytes bytes, 256-byte aligned, must outlive the lattice) and a
 * caller-owned HIP stream (hipStream_t, may be NULL for the null stream).
 * The populations are undefined until plbm_init_* or plbm_write_populations.
 * Errors: PLBM_E_INVALID, PLBM_E_NOMEM (dev_bytes too small),
 * PLBM_E_UNSUPPORTED (walls on an axis other than the last). */
int plbm_create(const plbm_lattice_desc* desc, const plbm_lattice_params* params, void* dev_mem,
                uint64_t dev_bytes, void* hip_stream, plbm_lattice** out);

/* f = f_eq(rho, u) (eq. Single_Phase_EDF) from host float64 fields rho[N] and
 * u[d][N] (u may be NULL: u = 0); resets time to 0.  Synchronises the stream. */
int plbm_init_fields(plbm_lattice* lat, const double* rho, const double* u);

/* f = f_eq of a density shape evaluated on the device; resets time to 0. */
int plbm_init_shape(plbm_lattice* lat, const plbm_shape* shape);

/* Enqueue n update steps on the lattice's stream and return without waiting.
 * One step is the update of Sec. II for every node: the pull of eq. (LBE),
 * density and momentum (eqs. Density, Momentum; u with F/2), psi (eq.
 * Interaction_Potential, float64 radicand), the force stencil (eq.
 * interactionForce), tau(rho) (Sec. VI), BGK or MRT collision with Guo forcing
 * (eqs. Single_Phase_EDF, Guo_Forcing_Scheme) and the store (periodic, or
 * half-way bounce-back walls on the last axis); or the well-balanced scheme of
 * the descriptor.  The first call (n = 0 included) captures replay graphs of
 * 16 and 2 steps; on a stream the caller is capturing, the launches go into
 * the caller's graph.  Errors: PLBM_E_INVALID (n < 0, lattice attached to a
 * batch), PLBM_E_DEVICE (a HIP error, its text in plbm_last_error). */
int plbm_step(plbm_lattice* lat, int64_t n);

/* rho[N] and u[d][N] at the current time (u includes F/2, eq. Momentum),
 * copied into host float64 buffers.  Synchronises the stream. */
int plbm_read_moments(plbm_lattice* lat, double* rho, double* u);

/* Same as plbm_read_moments into caller device buffers (float64), enqueued
 * on the lattice's stream without waiting. */
int plbm_moments_device(plbm_lattice* lat, void* rho_dev, void* u_dev);

/* Post-streaming populations f_i(x, t) at the current time, decoded to
 * float64, host layout f[q][...].  Synchronises the stream. */
int plbm_read_populations(plbm_lattice* lat, double* f);

/* Replace the state by host float64 populations f[q][...] (checkpoint
 * restore, fault injection).  Time is left unchanged.  Synchronises.
 * Locally shifted storage takes its reference densities from these
 * populations (two passes over f), so a read-write round trip is exact to
 * the storage rounding but not bitwise. */
int plbm_write_populations(plbm_lattice* lat, const double* f);

/* Steps taken since the last initialisation. */
int plbm_get_time(plbm_lattice* lat, int64_t* t);

/* Global diagnostics at the current time (the moments of eqs. Density and
 * Momentum, summed in a fixed order): compensated float64 mass, momentum,
 * max|u|, the residual max|u(t) - u(t-k)|/k against the u stored by the
 * previous reduction (k the steps since; u(t-k) kept in float32), and the
 * health flags; stores u for the next residual.  Synchronises the stream.
 * Returns PLBM_E_UNSTABLE (with *out filled) when the NaN or rho <= 0 flag is
 * raised. */
int plbm_reduce(plbm_lattice* lat, plbm_diag* out);

/* plbm_reduce for callers that cannot allocate device memory or have none to
 * spare for a workspace.  Same kernels, results and errors as plbm_reduce,
 * but the per-tile partial records and the final record live in a static
 * device array inside the library (2 MiB per GPU, held until the process
 * ends) instead of the lattice's buffer.  Allocates nothing.  The lattice's
 * device must be current.  Lattices of more than 32 767 tiles are refused
 * with PLBM_E_NOMEM (plbm_reduce has no such limit).  All calls on one GPU
 * share the array: calls that overlap in time on one GPU (several streams
 * or threads) race on it; serialise them. */
int plbm_reduce_static(plbm_lattice* lat, plbm_diag* out);

/* Release the handle (not the caller's device memory). */
void plbm_destroy(plbm_lattice* lat);

/* Continuous batching (a serving form; the paper has none): a batch step is
 * the update of plbm_step (Sec. II) for every attached lattice, and
 * plbm_batch_diag the reduction of plbm_reduce for each.  Attached lattices
 * may differ in size, lattice kind,
 * collision, storage, pattern, walls and scheme; those that share all six ("a
 * type") are advanced by one launch per step (two for the in-place pattern
 * and for the well-balanced scheme) whose workgroups cover the tiles of every
 * such slot, so each step costs one or two launches per type present.  max_slots
 * bounds the lattices attached at once and max_tiles their tiles together.
 * The batch owns no lattice memory; its work table lives in a caller-owned
 * device buffer of plbm_batch_bytes(max_slots, max_tiles) bytes and is
 * rewritten on the first step after an attach or detach.  plbm_batch_step(n)
 * enqueues n steps of every attached lattice on the batch's stream (runs of
 * 16 and 2 steps replayed from captured HIP graphs).  Results are bitwise identical
 * to stepping each lattice alone.  A lattice belongs to at most one batch at a
 * time: while attached, plbm_step, plbm_init_* and plbm_write_populations on
 * its own handle return PLBM_E_INVALID (reads stay allowed).  plbm_destroy of
 * an attached lattice detaches it first; plbm_batch_destroy releases every
 * lattice still attached.
 * Errors: PLBM_E_INVALID (bad slot, lattice attached to a batch already),
 * PLBM_E_NOMEM (dev_bytes too small, no free slot, more than max_tiles tiles). */
int plbm_batch_bytes(int32_t max_slots, int64_t max_tiles, uint64_t* bytes);
int plbm_batch_create(int32_t max_slots, int64_t max_tiles, void* dev_mem, uint64_t dev_bytes, void* hip_stream,
                      plbm_batch** out);
int plbm_batch_attach(plbm_batch* b, plbm_lattice* lat, int32_t* slot);
int plbm_batch_detach(plbm_batch* b, int32_t slot);
int plbm_batch_step(plbm_batch* b, int64_t n);
int plbm_batch_diag(plbm_batch* b, plbm_diag* per_slot); /* per_slot[max_slots]; unused slots zeroed */
void plbm_batch_destroy(plbm_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* PLBM_H */
