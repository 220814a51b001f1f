/*
 * cglbm.h -- C ABI of liblbm.so: the per-time-step update of the two-colour
 * D3Q27 colour-gradient lattice Boltzmann model with nonorthogonal central
 * moments (Saito, De Rosis, Festuccia, Kaneko, Abe, Koyama,
 * arXiv:1804.08923), on one AMD Instinct MI355X (gfx950).
 *
 * What a step computes (Sec. II of the paper):
 *   colour densities rho_k = sum_i f_i^k, order parameter phi (Eq. order),
 *   isotropic gradients of phi and rho, interpolated alpha_bar and nu_bar,
 *   body force F = (rho - rho_b0) g (Eq. bodyForceJet), velocity with the
 *   half-force term (Eq. Momentum), enhanced equilibrium (Eq. EES, Eq. Phi),
 *   GMRT central-moment collision and forcing (Eqs. scoll, ketF, ketFd) with
 *   s0 = s1 = 0 and s2b = s3 = s4 = s5 = s6 = 1, perturbation (Eq. perturb,
 *   Eq. B_i), recolouring (Eqs. op3r, op3b), streaming (Eq. LBE) and, for the
 *   jet problem, the inflow, free-slip and convective-outflow boundaries of
 *   Sec. IV A.
 *
 * Conventions shared by every entry point:
 *   - Lattice: nx*ny*nz nodes, node index n = (z*ny + y)*nx + x (x fastest).
 *     Directions i = 0..26 follow the paper's velocity set (Eq. velVec);
 *     with lattice == 19 (D3Q19, see lbm_params) i = 0..18, the same order
 *     without the eight corners.
 *   - Memory: the caller owns all device memory.  lbm_query_sizes() states
 *     the size of every buffer; the library stores the raw device pointers
 *     handed to lbm_init() and never allocates or frees device memory.
 *   - Streams: every call enqueues work on the stream given to lbm_init()
 *     (a hipStream_t passed as void*) and does not synchronise the host,
 *     except where a function says so.  One handle per stream; a handle is
 *     not thread-safe.
 *   - Errors: every function returns an int status (LBM_OK or a negative
 *     LBM_ERR_* code).  No exception crosses the ABI.  lbm_last_error()
 *     returns a thread-local message describing the last failure.
 */
#ifndef CGLBM_H
#define CGLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_ERR_INVALID_ARG (-1) /* a parameter or pointer failed validation */
#define LBM_ERR_UNSUPPORTED (-2) /* a valid request this library does not implement */
#define LBM_ERR_HIP (-3)         /* a HIP runtime call failed */
#define LBM_ERR_NONFINITE (-4)   /* the FP64 audit found a non-finite total */
#define LBM_ERR_STATE (-5)       /* call out of order (e.g. step before init) */

enum lbm_bc { LBM_BC_PERIODIC = 0, LBM_BC_JET = 1 };
/* Population storage (arithmetic is FP32 in every form; not in the paper):
 *   FP32     the colour-blind deviations d_i = f_i - w_i rho_b0 in FP32;
 *   BF16     the same deviations in bfloat16 (round to nearest even);
 *   FP16     the same deviations in IEEE binary16;
 *   BF16_EQ, FP16_EQ  equilibrium-referenced 16-bit forms: moving directions
 *            store d_i minus the phase and velocity parts of a per-node
 *            reference equilibrium (rho~, u~, rho kappa - rho_b0, rounded to
 *            the format and stored beside them), the rest population is
 *            kept exactly; slower, but the momentum no longer carries the
 *            16-bit rounding of the equilibrium. */
enum lbm_storage {
    LBM_STORAGE_FP32 = 0,
    LBM_STORAGE_BF16 = 1,
    LBM_STORAGE_FP16 = 2,
    LBM_STORAGE_BF16_EQ = 3,
    LBM_STORAGE_FP16_EQ = 4
};
enum lbm_init_kind {
    LBM_INIT_FIELDS = 0,  /* per-colour equilibria of caller fields rho_r, rho_b, u */
    LBM_INIT_DROPLET = 1, /* tanh droplet of Sec. III at rest */
    LBM_INIT_JET = 2      /* all blue at rest (Sec. IV A) */
};

/* Problem parameters in lattice units (c = delta_x = delta_t = 1). */
typedef struct lbm_params {
    int32_t nx, ny, nz;   /* lattice size; periodic: >= 1 each; jet: >= 3 each; each <= 65535;
                             (nx+2)(ny+2)(nz+2) <= 2^29 padded nodes */
    int32_t bc;           /* enum lbm_bc */
    int32_t storage;      /* enum lbm_storage: population storage format */
    int32_t init;         /* enum lbm_init_kind used by lbm_init */
    double rho_r0, rho_b0;/* reference densities; gamma = rho_r0 / rho_b0 (Sec. II) */
    double alpha_b;       /* alpha of the blue phase (the paper: 8/27); alpha_r = 1 - (1 - alpha_b)/gamma */
    double nu_r, nu_b;    /* kinematic viscosities (> 0); nu_bar is their phi-weighted harmonic mean */
    double A;             /* perturbation strength; sigma = (4/9) A tau (Eq. sigma) */
    double beta;          /* recolouring parameter in [0, 1] (the paper: 0.7) */
    double g[3];          /* gravity; the body force is (rho - rho_b0) g */
    double s_b, s3, s4, s5, s6; /* relaxation rates of the bulk and higher moments: must be 1 */
    double grad_eps;      /* |grad phi| <= grad_eps switches perturbation and recolouring term off */
    /* jet inlet (bc == LBM_BC_JET): circle (x - cx)^2 + (y - cy)^2 < (D/2)^2 at z = -1/2 */
    double inlet_cx, inlet_cy, inlet_D, inlet_u;
    double noise_amp;     /* radial inlet velocity noise amplitude, fraction of inlet_u */
    uint64_t noise_seed;  /* seed of the counter-based SplitMix64 noise */
    /* droplet preset (init == LBM_INIT_DROPLET): centre, radius, interface width W */
    double drop_cx, drop_cy, drop_cz, drop_R, drop_W;
    /* velocity set: 27 (or 0) the paper's D3Q27; 19 the reduced D3Q19 lattice
       that Sec. II and Sec. IV B suggest to cut the cost, with coefficients
       derived by keeping every moment the D3Q27 ones fix: weights 1/3, 1/18,
       1/36; varphi_i = alpha at rest and 1.5 w_i (1 - alpha) otherwise (so
       alpha_b = 1/3 gives c_s^2 = 1/3); Phi_i = -3 nu_bar u.grad rho at rest and
       m_i nu_bar (c.u)(c.grad rho)/4 with m = 2 (faces), 1 (edges); B_i = -1/3
       at rest and w_i otherwise; the 19 rows of Eq. momentSet that are
       independent on D3Q19.  D3Q19 supports both boundary kinds (the jet with
       the same inlet, free-slip and outflow rules), FP32 storage only (else
       LBM_ERR_UNSUPPORTED), the three presets, at most 2^31 nodes, and the
       entry points lbm_query_sizes, lbm_init,
       lbm_step, lbm_macroscopic, lbm_get_state, lbm_set_state, lbm_time,
       the jet diagnostics (both forms), lbm_profile, lbm_profile_read and
       lbm_destroy; the snapshot and adjoint calls return
       LBM_ERR_UNSUPPORTED.  Q below is 27,
       or 19 for D3Q19. */
    int32_t lattice;
    int32_t lattice_pad;  /* unused */
} lbm_params;

/* Byte sizes of the caller-allocated device buffers. */
typedef struct lbm_sizes {
    uint64_t n_nodes;
    uint64_t pop_bytes;     /* each of the two population buffers (A and B): 54 planes of
                               (nx+2)(ny+2)(nz+2) padded nodes in the storage format
                               (D3Q19: the larger of 39 planes of N floats, the form
                               init and set_state write, and the 19 planes plus a 16-byte
                               record per node that a step writes) */
    uint64_t field_bytes;   /* per-node fields and recolouring scalars: 11 floats per padded node
                               (19 with the reference records of BF16_EQ / FP16_EQ; D3Q19:
                               4 floats per node) */
    uint64_t hist_bytes;    /* outlet planes of the previous and current step, 2 x 54 floats
                               per (x, y) (D3Q19: 2 x 38); jet only */
    uint64_t audit_bytes;   /* FP64 partial sums of the audit reduction */
    uint64_t inlet_bytes;   /* optional inlet axial-velocity profile, nx*ny floats */
    uint64_t adjoint_bytes; /* adjoint work buffer (see lbm_adjoint_step) */
    uint64_t state_bytes;   /* a full FP32 state: 2Q floats per node (fr[Q], fb[Q]) */
    uint64_t snap_bytes;    /* one state snapshot in the library's own layout (see lbm_step_into):
                               27 population planes of (nx+2)(ny+2)(nz+2) padded nodes in the
                               storage format (28 for BF16_EQ / FP16_EQ), a 16-byte record per
                               padded node (two for BF16_EQ / FP16_EQ), and for the jet one
                               outlet plane of 54 floats per (x, y): about 124 B per node in FP32 */
} lbm_sizes;

/* Device buffers owned by the caller; must stay valid until lbm_destroy(). */
typedef struct lbm_buffers {
    void* pop_a;             /* pop_bytes, 256-byte aligned */
    void* pop_b;             /* pop_bytes, 256-byte aligned */
    float* fields;           /* field_bytes, 16-byte aligned */
    float* hist;             /* hist_bytes; may be NULL when bc == LBM_BC_PERIODIC */
    double* audit;           /* audit_bytes */
    const float* inlet_uz;   /* NULL: uniform inlet_u; else nx*ny axial velocities (x fastest) */
    void* adjoint;           /* adjoint_bytes, 256-byte aligned, or NULL if lbm_adjoint_step is never called */
} lbm_buffers;

typedef struct lbm_handle lbm_handle;

/* Fill *out with the buffer sizes for p.  Validates p (LBM_ERR_INVALID_ARG /
 * LBM_ERR_UNSUPPORTED as lbm_init). */
int lbm_query_sizes(const lbm_params* p, lbm_sizes* out);

/* Create a handle and write the initial state (time t = 0) into buf->pop_a.
 * With p->init == LBM_INIT_FIELDS the populations are the per-colour
 * equilibria f_i^k = rho_k {varphi_i(alpha_k) + w_i [velocity terms of
 * Eq. EES]} of the device fields rho_r[n], rho_b[n] and u[3n..3n+2] (float,
 * node order; u may be NULL for rest).  The presets ignore the three field
 * pointers: the droplet of Sec. III (rho_k = rho_k0/2 [1 -/+ tanh(2(r-R)/W)])
 * or the all-blue jet domain at rest.  Validation rejects nu <= 0,
 * rho0 <= 0, alpha_b outside (0, 1), alpha_r outside [0, 1), beta outside
 * [0, 1], rates s_b..s6 != 1 (LBM_ERR_UNSUPPORTED), a jet lattice smaller
 * than 3 in any dimension or an inlet circle that touches the side walls,
 * NULL or misaligned buffers.  Writes *h = NULL on failure. */
int lbm_init(lbm_handle** h, const lbm_params* p, const lbm_buffers* buf,
             const float* rho_r, const float* rho_b, const float* u, void* hip_stream);

/* Enqueue n_steps full time steps.  Never synchronises the host. */
int lbm_step(lbm_handle* h, int32_t n_steps);

/* Macroscopic fields of the current state into caller device arrays (each may
 * be NULL): rho_r[n], rho_b[n], u[3n + a] with the F/2 term of Eq. Momentum,
 * phi[n] (Eq. order).  If audit (HOST pointer, 5 doubles) is not NULL the
 * call also computes the FP64 totals sum rho_r, sum rho_b, sum rho u_x,
 * sum rho u_y, sum rho u_z, synchronises the stream, and returns
 * LBM_ERR_NONFINITE if any total is not finite. */
int lbm_macroscopic(lbm_handle* h, float* rho_r, float* rho_b, float* u, float* phi,
                    double* audit);

/* Copy the current state (time lbm_time()) into a device array of
 * state_bytes: fr[i*N + n] for i < Q, then fb[i*N + n] (the populations
 * after streaming, Q = 27 or 19 by p->lattice). */
int lbm_get_state(lbm_handle* h, float* state);

/* Replace the current state by a device array in the lbm_get_state layout
 * and set the time level to t (the inlet noise depends on it).  For the jet
 * the outlet history becomes the outlet plane of this state. */
int lbm_set_state(lbm_handle* h, const float* state, int64_t t);

/* Time level of the current state (number of steps since init or the t of
 * the last lbm_set_state / lbm_snapshot_load). */
int64_t lbm_time(const lbm_handle* h);

/* State snapshots: the state between two steps in the library's own layout
 * (the colour-blind deviations as the last step streamed them, the per-node
 * recolouring records that rebuild both colours, Eqs. op3r/op3b, and the
 * jet's outlet plane of Sec. IV A), for checkpointing a run whose gradient
 * is taken with lbm_adjoint_step_snapshot.  A snapshot is snap_bytes of
 * caller-owned device memory, 256-byte aligned; the library keeps no pointer
 * to it except as stated for lbm_step_into.  A snapshot is only meaningful
 * for the handle (parameters and storage) that wrote it.
 *
 * lbm_step_into: one full time step (as lbm_step) whose result is written
 *   into snap instead of the handle's own buffers; snap then IS the current
 *   state (time + 1) and is read in place by the next call that reads the
 *   state (lbm_step, lbm_macroscopic, lbm_get_state, lbm_snapshot_save, ...),
 *   so it must stay valid and unmodified until the next lbm_step,
 *   lbm_step_into, lbm_set_state or lbm_snapshot_load.  snap must not be the
 *   current state itself (LBM_ERR_INVALID_ARG).  This is the recompute of a
 *   checkpointed segment at the cost of a forward step.
 * lbm_snapshot_save: copy the current state into snap (device copies on the
 *   stream).  LBM_ERR_STATE right after lbm_init or lbm_set_state, whose
 *   general state has no snapshot form (take one step first, or keep the
 *   lbm_get_state array).
 * lbm_snapshot_load: make a copy of snap the current state, at time level t
 *   (the inlet noise depends on it); the handle's own buffers receive it. */
int lbm_step_into(lbm_handle* h, void* snap);
int lbm_snapshot_save(lbm_handle* h, void* snap);
int lbm_snapshot_load(lbm_handle* h, const void* snap, int64_t t);

/* One reverse (adjoint) step of the time step t -> t+1 (not in the paper:
 * the hand-written reverse mode of every operation listed at the top of
 * this file, including the jet boundaries).
 *   state_t    device, lbm_get_state layout: the forward state at time t
 *              (the caller recomputes it, e.g. from a checkpoint);
 *   t          its time level (the inlet noise depends on it);
 *   lambda_in  device, same layout: cotangent of the state at t+1;
 *   lambda_out device, same layout, written: (d x_{t+1} / d x_t)^T lambda_in;
 *              must not alias lambda_in or state_t;
 *   dJ_dA      device, 1 double, incremented by lambda_in . d x_{t+1}/dA;
 *   dJ_du_in   device, nx*ny floats or NULL; jet only: incremented by
 *              lambda_in . d x_{t+1}/d u_in, u_in the inlet axial-velocity
 *              profile (entries outside the inlet circle stay unchanged).
 * The step is differentiated in exact arithmetic: the rounding of the
 * population storage format is not modelled, so any storage works.  At the
 * non-differentiable points (|grad phi| = grad_eps, u_z = 0 in the outflow
 * condition) the one-sided derivative of the branch taken is used.  Needs
 * buf->adjoint (adjoint_bytes); overwrites the per-node field scratch that
 * every lbm_step recomputes, and leaves the populations and the time level
 * of the handle unchanged.  Enqueued on the handle's stream; no host sync. */
int lbm_adjoint_step(lbm_handle* h, const float* state_t, int64_t t, const float* lambda_in,
                     float* lambda_out, double* dJ_dA, float* dJ_du_in);

/* The same reverse step with the forward state x_t given as a snapshot
 * (device, snap_bytes, written by lbm_step_into or lbm_snapshot_save of this
 * handle at time level t) instead of the 54-plane FP32 array.  Arguments,
 * outputs and error behaviour as lbm_adjoint_step; lambda_out must not
 * alias lambda_in or snap_t.  The forward quantities are rebuilt from the
 * snapshot exactly as the next lbm_step would read it. */
int lbm_adjoint_step_snapshot(lbm_handle* h, const void* snap_t, int64_t t, const float* lambda_in,
                              float* lambda_out, double* dJ_dA, float* dJ_du_in);

/* Instrumentation: with enable != 0, lbm_step records HIP events on its
 * stream around its kernel groups (density pass; fused collide-recolour-
 * stream kernel; boundary kernels: ghost-shell fills);
 * enable == 0 stops recording. */
int lbm_profile(lbm_handle* h, int enable);

/* Synchronise on the last recorded event, return the summed time in
 * milliseconds and the number of recorded steps since the last read for the
 * density pass (index 0), the fused kernel (index 1) and the boundary kernels
 * (index 2), and clear them. */
int lbm_profile_read(lbm_handle* h, double* ms /* 3 */, int64_t* launches /* 3 */);

/* Jet diagnostics of Sec. IV C on the current state (not part of a step;
 * readings: the jet phase is phi > 0, components are face-connected without
 * wrap-around, volumes count nodes).
 *   jet_nodes      nodes with phi > 0 (phi as lbm_macroscopic returns it);
 *   front_z        the leading edge: largest z of a jet node, -1 if none;
 *   column_volume  nodes of the components with a node on the inlet plane
 *                  z = 0 (the continuous column from the nozzle);
 *   n_fragments    the other components, the fragments; their equivalent
 *                  diameters are d = (6 V / pi)^(1/3) of their volumes V. */
typedef struct lbm_jet_stats {
    int64_t jet_nodes;
    int64_t front_z;
    int64_t column_volume;
    int64_t n_fragments;
} lbm_jet_stats;

/* Bytes of the device work buffer lbm_jet_diagnostics needs (16 per node
 * plus a 256-byte header). */
int lbm_diag_bytes(const lbm_params* p, uint64_t* bytes);

/* Compute the jet diagnostics of the current state.
 *   work     device, lbm_diag_bytes() bytes, 256-byte aligned, caller-owned
 *            (contents on entry do not matter; overwritten);
 *   stats    HOST, filled;
 *   volumes  HOST, cap entries (may be NULL when cap == 0): the volumes of
 *            the first min(n_fragments, cap) fragments, in no particular
 *            order.
 * Enqueued on the handle's stream; synchronises the host before returning.
 * Connected components come from a lock-free union-find (atomic minimum on
 * parent indices); the result does not depend on the order of the atomics. */
int lbm_jet_diagnostics(lbm_handle* h, void* work, lbm_jet_stats* stats, int64_t* volumes, int64_t cap);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * diagnostics as lbm_jet_diagnostics, with the work memory taken from a
 * static array of the library instead of a caller buffer.  The array holds
 * the work of at most 2^22 nodes (64 MiB + 256 B); it exists once on every
 * GPU the library runs on, from the first lbm_init on that GPU until the
 * process ends.  Larger lattices: LBM_ERR_UNSUPPORTED.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the host
 * copies go straight into stats and volumes.  All calls on one GPU share
 * that GPU's array, and the last call's contents remain in it: calls that
 * overlap in time on one GPU (other threads, other streams, other handles)
 * race and must be serialised by the caller.  Arguments, results and the
 * host synchronisation are those of lbm_jet_diagnostics. */
int lbm_jet_diagnostics_static(lbm_handle* h, lbm_jet_stats* stats, int64_t* volumes, int64_t cap);

/* Release the handle (not the caller's buffers).  NULL is accepted. */
int lbm_destroy(lbm_handle* h);

/* Static description of a status code. */
const char* lbm_status_string(int status);

/* Thread-local message of the last failure in this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CGLBM_H */
