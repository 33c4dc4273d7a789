/*
 * rmrt.h -- C ABI of the MI355X (gfx950) rectangular multiple-relaxation-time
 * lattice Boltzmann library (RMRT-LB of Chai, Yuan & Shi, arXiv:2206.00366).
 *
 * One call of rmrt_step advances every node by the evolution equation in its
 * moment-space form (Sec. V eq. 2-2-3, with fbar = f - dt F / 2 of Sec. II
 * eq. 2-3): raw moments m = M fbar (eq. 5-2), relaxation with the block
 * relaxation matrix S whose second-order block comes from the shear and bulk
 * viscosities (Sec. IV eq. 4-27, 4-31; Sec. V eq. 5-8), back-transform
 * M^-1 (eq. 5-4), then propagation f(x + c_j dt) (Sec. II eq. 2-2).
 *
 * Conventions shared by every entry point
 *   - Lattice units: c_a = dx_a / dt.  Nodes are indexed x-fastest:
 *     node = x + nx * (y + ny * z); 2D problems use nz = 1.
 *   - Population buffers are structure-of-arrays: slot j of node i lives at
 *     element j * ld + i, j in the paper's velocity order (rD2Q9 eq. 3-1,
 *     rD3Q27 eq. 3-2; rD3Q19 = first 19 of rD3Q27; rD2Q5 / rD3Q7 = first
 *     5 / 7).  The stream stride ld >= N = nx*ny*nz is the library's choice
 *     for N and the storage: size buffers with rmrt_population_bytes
 *     (= q * ld * element size); elements [j ld + N, (j + 1) ld) are padding
 *     that no call reads or writes.
 *   - Stored values are deviations from the rest equilibrium:
 *       RMRT_F64    : double  d_j = fbar_j - w_j rho0
 *       RMRT_F32DEV : float   d_j = fbar_j - w_j rho0
 *       RMRT_F16DEV : _Float16 h_j = (fbar_j - w_j rho0) / w_j  (round to nearest even)
 *     (rho0 is the reference density of the NSE, or the reference phi of the
 *     NCDE, usually 0.)
 *   - Every device pointer is caller-owned device memory borrowed for the
 *     lifetime of the context; the library owns only the context, its device
 *     parameter block, reduction scratch and any captured graph.
 *   - Every call is ordered on the caller's hipStream_t (passed as void*;
 *     NULL = the default stream).  Only rmrt_reduce and rmrt_residual
 *     synchronise that stream, to return their FP64 results to the host.
 *   - Every function returns RMRT_OK (0) or a negative RMRT_E* code; a
 *     thread-local message is available from rmrt_last_error().  Nothing
 *     throws across the ABI.
 */
#ifndef RMRT_H
#define RMRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define RMRT_OK 0
#define RMRT_EINVAL (-1)        /* invalid argument or parameter set            */
#define RMRT_EUNSUPPORTED (-2)  /* valid but not built (e.g. Q9 with nz > 1)    */
#define RMRT_EHIP (-3)          /* a HIP runtime call failed                    */
#define RMRT_ENONFINITE (-4)    /* a reduction found NaN or Inf                 */
#define RMRT_ENOMEM (-5)        /* host or device allocation failed             */

/* ---- enumerations ---- */
enum { RMRT_Q9 = 0, RMRT_Q19 = 1, RMRT_Q27 = 2, RMRT_Q5 = 3, RMRT_Q7 = 4 };
/* rD2Q9, rD3Q19, rD3Q27 (Sec. III); rD2Q5 (the rD2Q5I subset) and rD3Q7 with
 * the weights of Remark I of Sec. III carry the NCDE only, in the C = 0 form
 * of eq. 4-16: linear equilibrium g_eq(phi, phi adv, 0), F_j = w_j S and
 * G_j = g_eq(0, (1 - s_1/2) dB/dt, 0) with dB/dt = adv (phi - phi_prev) / dt
 * from the previous step's phi, which the context keeps in a library-owned
 * field of N doubles (FP64 storage) or floats (else); rmrt_init and
 * rmrt_set_fields set it to the initial phi (dB/dt = 0 on the first step). */
enum { RMRT_NSE = 0, RMRT_NCDE = 1 };                              /* Sec. IV B / IV A      */
enum { RMRT_F64 = 0, RMRT_F32DEV = 1, RMRT_F16DEV = 2 };           /* population storage    */
enum { RMRT_AB = 0, RMRT_AA = 1 };                                 /* two-lattice / in-place */
enum { RMRT_OUT_F64 = 0, RMRT_OUT_F32 = 1 };                       /* macroscopic outputs   */

/* wall_faces bits: 1 = halfway bounce-back wall on that face, 0 = periodic */
#define RMRT_WALL_XM 1u
#define RMRT_WALL_XP 2u
#define RMRT_WALL_YM 4u
#define RMRT_WALL_YP 8u
#define RMRT_WALL_ZM 16u
#define RMRT_WALL_ZP 32u

/*
 * Parameters of one rectangular domain.  The notes below give, per field, the
 * values that select its documented default: dt, cs2 and s_hi take theirs at
 * zero, nu_b and w_corner only when negative (a zero bulk viscosity is
 * rejected, a zero corner weight is valid).
 *
 *   lattice, equation, storage, pattern : enumerations above (FP16
 *             deviation storage needs every weight > 0)
 *   n[3]      nodes per axis (n[2] = 1 for rD2Q9 and rD2Q5)
 *   dx[3]     grid spacings dx_a; dt time step (<= 0 -> 1)          (Sec. III)
 *   cs2       sound speed squared c_s^2 (<= 0 -> min_a c_a^2 / 3); must satisfy
 *             0 < c_s^2 / c_a^2 < 1 (eq. 3-3-3 / eq. 3-3-8 bounds)
 *   nu, nu_b  kinematic shear and bulk viscosity (NSE; nu_b < 0 -> 2 nu / d,
 *             which makes the second-order block diagonal, Remark V of Sec. IV)
 *   s_hi      rate of every moment of order >= 3 (NSE, <= 0 -> s_nu) or >= 2
 *             (NCDE, <= 0 -> 1); these rates do not enter the recovered PDE
 *   w_corner  rD3Q27 omega_19 (< 0 -> r1 r2 r3 / 8, r_a = c_s^2 / c_a^2)
 *   D0, D2    NCDE diffusivity D(phi) = D0 (1 + D2 phi^2); K = D(phi) I
 *             through the local first-order rate (eq. 4-10, beta = 1)
 *   adv[3]    NCDE constant advection velocity: B = phi adv (eq. NCDE)
 *   force[3]  NSE body-force density Fbar (eq. NSE), constant in space
 *   source    NSE mass source Sbar, or NCDE source S, constant in space
 *   rho0      reference density (NSE) or reference phi (NCDE) of the stored
 *             deviations
 *   wall_faces RMRT_WALL_* bits (halfway bounce-back); other faces periodic
 *   check_every if > 0, rmrt_step runs an FP64 mass check every that many
 *             steps and returns RMRT_ENONFINITE when it is not finite
 *   incompressible  NSE: 1 selects the He-Luo equilibrium
 *             g_eq(rho, rho0 u, rho0 u u) with rho0 u = sum_j c_j f_j (Sec. V,
 *             eq. meqd2q9-HL; Remark IV of Sec. IV); rmrt_moments then returns
 *             u = sum_j c_j f_j / rho0.  0 = the equilibrium of eq. NSEfeq.
 *   nu_tensor[6]  NSE: viscosity tensor entries of eq. 4-29, in the order
 *             (xx, yy, zz, xy, xz, yz): K_mu,aa = rho nu_tensor[a] sets s_s,a and
 *             K_mu,ab = rho nu_tensor[ab] sets s_ab (eq. 4-31 per entry);
 *             entries <= 0 take nu (the isotropic case)
 *   gamma0    NCDE: 1 selects the gamma = 0 form of eq. 2-1, in which the
 *             dt^2/2 dF/dt term is the explicit difference of F (zero for the
 *             constant source S): populations are f itself (no fbar = f -
 *             dt F / 2 transform), phi = sum_j f_j, and the source enters as
 *             dt F instead of dt (I - Lambda/2) F.  0 = the gamma = 1 form
 *             (eq. 2-3), the only one for the NSE.
 *   diffusive NCDE: 1 selects the diffusive-scaling model of eq. 4-17: the
 *             dt^2/2 D F term removed (populations f, phi = sum f, as gamma0),
 *             f_eq = g_eq(phi, phi adv, 0) (C = 0) and G = 0
 *   nu_b_axis[3]  NSE: per-axis bulk viscosities K_mu_b,aa = rho nu_b_axis[a]
 *             of eq. 4-29 (set s_b,a); entries <= 0 take nu_b (a zero-initialised
 *             struct is the isotropic model)
 *   c_zero    NCDE on rD2Q9 / rD3Q19 / rD3Q27: 1 selects the C = 0 form of
 *             eq. 4-16 (the second branch of eq. 4-11): f_eq = g_eq(phi, phi adv, 0)
 *             and G_j = g_eq(0, (1 - s_1/2) dB/dt, 0) with dB/dt = adv (phi -
 *             phi_prev) / dt from the previous step's phi, kept in a
 *             library-owned field as on rD2Q5 / rD3Q7 (which always take
 *             this form); 0 = C = phi adv adv (the first branch)
 *   central   NSE on rD2Q9 / rD3Q27: 1 relaxes in the central moments
 *             kappa = N(u) M fbar (the cascaded basis of eq. 5-1-1, N(u) the
 *             binomial shift by the node's u) with the same relaxation blocks
 *             as the raw-moment model (full second-order block from nu, nu_b;
 *             s_ab; s_hi above) and the equilibrium, auxiliary and source
 *             moments shifted alike, so Lambda = M^-1 N^-1 S N M (eq. 5-1-2);
 *             the recovered NSE is the same, the higher moments relax in the
 *             frame moving with the fluid.  RMRT_EUNSUPPORTED on the other
 *             lattices; local outputs are refused with it.
 *   hermite   NSE on rD2Q9 / rD3Q19 / rD3Q27: 1 relaxes in the Hermite
 *             moments H M fbar, the tensor products of H_0 = 1, H_1 = xi,
 *             H_2 = xi^2 - cs2 of each velocity (eq. 5-1-1 with the constant
 *             lower-triangular N = H), with the raw model's blocks and every
 *             moment vector transformed alike (eq. 5-1-2); with central = 1
 *             the central-Hermite moments H N(u) M fbar (xi = c - u).  Local
 *             outputs are refused with it.
 *   bhll      NSE on rD2Q9: 1 relaxes in the orthogonal BHLL moments
 *             N_BHLL M_a fbar (Sec. V, eq. Md2q9-2 / Md2q9-3, a = c_y / c_x,
 *             M_a the raw moments of the velocities in units of c_x), each
 *             order on its own with that order's block of N S N^-1: the
 *             second-order block of eq. 5-8 carried over by similarity, s_ab on
 *             p_xy, s_hi on q_x, q_y and epsilon (eq. 5-1-2).  RMRT_EINVAL
 *             with central or hermite, RMRT_EUNSUPPORTED on the other
 *             lattices; local outputs are refused with it.
 */
typedef struct rmrt_params {
  int lattice, equation, storage, pattern;
  int n[3];
  double dx[3];
  double dt;
  double cs2;
  double nu, nu_b, s_hi;
  double w_corner;
  double D0, D2;
  double adv[3];
  double force[3];
  double source;
  double rho0;
  unsigned wall_faces;
  int check_every;
  int incompressible;
  double nu_tensor[6];
  double nu_b_axis[3];
  int gamma0;
  int diffusive;
  int c_zero;
  int central;
  int hermite;
  int bhll;
} rmrt_params;

/* Values the library derives from a parameter set (host only, no GPU). */
typedef struct rmrt_derived {
  int q, d;
  double c[3], cs2;
  double w[27];           /* weights, paper order (eq. 3-3-5, eq. 3-3-8)          */
  double s_nu, s_s[3], s_b[3], s_hi;  /* rates from eq. 4-31                      */
  double Sbar2[3][3];     /* second-order diagonal block, eq. 5-8-1                */
  double nu_b;
  double s_pair[3];       /* off-diagonal second-order rates (xy, xz, yz), eq. 4-31 */
} rmrt_derived;

typedef struct rmrt_ctx rmrt_ctx;
typedef struct rmrt_batch rmrt_batch;

/* Thread-local message of the last failing call ("" if none). */
const char* rmrt_last_error(void);

/* Library version string. */
const char* rmrt_version(void);

/*
 * HBM bandwidth probe (not part of the method): copies `bytes` (a multiple of
 * 16) from src to dst on stream with 16-byte vector loads and stores.  Used to
 * measure the achievable copy ceiling next to the lattice kernels.
 */
int rmrt_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/*
 * Validate a parameter set and fill *out with the derived lattice weights and
 * relaxation rates (Sec. III eq. 3-3-5 / 3-3-8; Sec. IV eq. 4-31; Sec. V
 * eq. 5-8-1).  Host only.  Returns RMRT_EINVAL for: an unknown enumeration,
 * n < 1, rD2Q9 with n[2] != 1, dx <= 0, c_s^2 >= c_a^2 on any axis, a negative
 * weight, nu <= 0 or nu_b <= 0 (NSE), D0 <= 0 (NCDE) or a rate outside (0, 2).
 */
int rmrt_derive(const rmrt_params* p, rmrt_derived* out);

/* Bytes of one population buffer for p (q * ld * element size, ld >= N the
 * stream stride above). Host only. */
int rmrt_population_bytes(const rmrt_params* p, size_t* bytes);

/*
 * Create a context for one domain and write the initial populations.
 *   f0, f1  device population buffers (rmrt_population_bytes each); f1 must be
 *           NULL for RMRT_AA and non-NULL for RMRT_AB
 *   solid   device uint8 mask of N nodes (1 = solid, bounce-back), or NULL
 *   rho     device double[N]: initial rho (NSE) or phi (NCDE)
 *   u       device double[d*N] SoA initial velocity (NSE; ignored by the NCDE)
 *   with_fne 1 adds the non-equilibrium part g_eq(0, 0, m_2^ne) built from the
 *           central-difference velocity gradient (Sec. IV eq. fne, eq. 4-34)
 * The initial state is fbar = f_eq(rho, u) - dt F / 2 [+ f_ne] (eq. NSEfeq,
 * eq. NSEFeq, eq. 2-3).  Asynchronous on stream.
 */
int rmrt_init(rmrt_ctx** out, const rmrt_params* p, void* f0, void* f1, const uint8_t* solid,
              const double* rho, const double* u, int with_fne, void* stream);

/* Re-initialise the populations of an existing context (same meaning as in rmrt_init). */
int rmrt_set_fields(rmrt_ctx* ctx, const double* rho, const double* u, int with_fne, void* stream);

/*
 * Source and force fields that vary from node to node (eq. NSE: mass source
 * Sbar(x) and body-force density Fbar(x); eq. NCDE: source S(x)), in place of
 * the constant source and force of the parameter set, which are then ignored.
 *   S  device array of N values: Sbar (NSE) or S (NCDE); NULL = zero
 *   F  device array of d*N values, SoA (component a of node i at a*N + i):
 *      Fbar (NSE only; RMRT_EINVAL for the NCDE); NULL = zero
 * Element type: double for RMRT_F64 storage, float otherwise.  Both NULL
 * detaches the fields (the constants apply again).  The arrays are borrowed:
 * every step reads the values they hold when it runs, so the caller may
 * change them between steps (stream-ordered) for sources that vary in time;
 * the steps of one multi-step call (one graph) see the same values.
 * Every formula takes the node's value: rho = sum fbar + dt Sbar/2, u =
 * (sum c fbar + dt Fbar/2) / rho (eq. 2-4-2), F_j = g_eq(Sbar, Fbar, -cs2 Sbar
 * I) and M_2G (eq. NSEFeq, M2GComput a); phi = sum fbar + dt S/2 (eq. 2-4-1),
 * F_j = w_j S (eq. 4-14-1).  In the gamma = 0 NCDE form (gamma0 = 1, eq. 2-1)
 * the step adds dt (F(t) - F(t - dt)) / 2 with F(t - dt) the source the
 * previous step read, kept by the library in a field of N values that this
 * call allocates and sets to S (the first step sees no difference).  The
 * initial state of rmrt_init / rmrt_set_fields (fbar = f_eq - dt F/2) takes
 * the fields attached at that time: attach, then (re)initialise.
 * Extra algorithmic bytes per update: one read of S (and d of F for the NSE)
 * in the working precision; with gamma = 0 one more read and one write.
 * Local outputs (rmrt_local_gradients, rmrt_step_local) return
 * RMRT_EUNSUPPORTED while fields are attached; RMRT_EINVAL on a domain of a
 * batch.  Drops the context's cached graphs; synchronises stream.
 */
int rmrt_set_source_fields(rmrt_ctx* ctx, const void* S, const void* F, void* stream);

/*
 * Advance nsteps >= 0 time steps (eq. 2-2-3 then propagation with halfway
 * bounce-back).  nsteps > 1 replays a HIP graph of nsteps launches that is
 * captured on first use and cached per (nsteps, parity).
 */
int rmrt_step(rmrt_ctx* ctx, int nsteps, void* stream);

/*
 * Capture, instantiate and upload (on stream) the graphs that
 * rmrt_step(ctx, nsteps) will replay from the context's current step count,
 * without running them or advancing the state.  Optional: rmrt_step captures
 * a graph on its first use; calling this first keeps the capture out of a
 * timed region or a latency-sensitive loop.  RMRT_EINVAL for a domain of a
 * batch or nsteps < 0.
 */
int rmrt_step_prepare(rmrt_ctx* ctx, int nsteps, void* stream);

/*
 * Macroscopic fields of the current state (eq. 2-4-1 / eq. 2-4-2):
 * rho (or phi) into rho_out[N]; u into u_out[d*N] SoA (may be NULL).
 * out_dtype RMRT_OUT_F64 or RMRT_OUT_F32.  Solid nodes are written as rho0, 0.
 */
int rmrt_moments(rmrt_ctx* ctx, void* rho_out, void* u_out, int out_dtype, void* stream);

/* Decode the current state into full populations fbar_j (double, q*N, natural layout). */
int rmrt_populations(rmrt_ctx* ctx, double* f_out, void* stream);

/*
 * Local derivative outputs of the current state, from the non-equilibrium
 * moments of each node alone (no finite differences), computed in FP64:
 *   RMRT_GRAD_STRESS (NSE): the generalized shear stress of eq. 4-32-0,
 *     tau = -(I - S_2/2) [sum_k c_k c_k f_k^ne + dt/2 (u F + F u + (cs2 I - u u) S)]
 *     with the full second-order relaxation block S_2 of eq. 4-27;
 *   RMRT_GRAD_STRAIN (NSE): the strain rate (grad u + grad u^T) / 2 from tau
 *     through eq. 4-28 with K_mu = rho nu I and K_mu_b = rho nu_b I (eq. 4-31);
 *   RMRT_GRAD_PHI (NCDE): grad phi from eq. 4-13 with D = phi I, K = D(phi) I:
 *     -D(phi) grad phi = (1 - s_1/2) (sum_k c_k f_k^ne + dt/2 X), X = adv S,
 *     or adv (phi - phi_prev) / dt on rD2Q5 / rD3Q7 (eq. 4-16).
 * out: device array (double, or float with RMRT_OUT_F32) of ncomp * N values,
 * component k of node i at out[k * N + i]; ncomp = 3 (xx, yy, xy) in 2D and 6
 * (xx, yy, zz, xy, xz, yz) in 3D for stress and strain, d for grad phi.
 * Solid nodes get zeros.  RMRT_EINVAL for a kind that does not match the
 * equation.  Accuracy: the stress scheme is exact for steady plane shear and
 * carries O(Ma) compressibility errors; the grad phi scheme carries an error
 * of first order in |adv|.
 */
#define RMRT_GRAD_STRAIN 0
#define RMRT_GRAD_STRESS 1
#define RMRT_GRAD_PHI 2
int rmrt_local_gradients(rmrt_ctx* ctx, int kind, void* out, int out_dtype, void* stream);

/*
 * One step fused with the local outputs of rmrt_local_gradients (same kinds,
 * layout, errors and zeros at solid nodes): out receives the output of the
 * state the step starts from, computed from the deviations the step has
 * loaded, in the step's working precision (FP64 for FP64 storage, FP32
 * otherwise), so the second non-equilibrium moment carries the FP32 rounding
 * of the collision.  Costs one step plus the output writes (no second read of
 * the state).  Advances the context by one step (one workgroup per tile, the
 * context's residency cap and tile order, 64-bit addressing; no health check).  RMRT_EINVAL
 * for a domain of a batch.  For the coupling loops of eq. 4-28 (a strain-rate
 * dependent viscosity) and eq. 4-13.
 */
int rmrt_step_local(rmrt_ctx* ctx, int kind, void* out, int out_dtype, void* stream);

/*
 * FP64 sums over fluid nodes: out[0] = sum rho (or phi), out[1..3] = sum rho u
 * (eq. 2-4-2; the mass and momentum that eq. 4-18-1 conserves).  Synchronises
 * stream.  Returns RMRT_ENONFINITE if any sum is NaN or Inf.
 */
int rmrt_reduce(rmrt_ctx* ctx, double out[4], void* stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the sums of rmrt_reduce
 * (same kernels, same summation order, same values) written to out[0..3],
 * caller-owned DEVICE memory (4 doubles), asynchronously on stream, with no
 * host synchronisation, no allocation and no memset, so the call can be
 * captured into a graph.  The block partial sums live in one fixed file-scope
 * device array of the library (2048 x 5 doubles = 80 KiB per GPU, held until
 * the process ends); the reduction launches at most 2048 workgroups whatever
 * the domain size, and RMRT_EINVAL reports a launch that would need more.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (concurrent streams, or host threads) race and must be serialised by the
 * caller; consecutive calls on one stream are safe.  Like every captured
 * launch of this library, a captured call reads the state in the layout of
 * the step count at capture time (the AA parity).  Finiteness is not
 * checked (the host never sees the values); RMRT_EINVAL for a NULL argument,
 * RMRT_EHIP if the array's device address cannot be obtained.
 */
int rmrt_reduce_noalloc(rmrt_ctx* ctx, double* out, void* stream);

/*
 * Steady-state residual r = ||u^n - u^prev||_2 / ||u^n||_2 (FP64, fluid nodes)
 * against the velocity stored by the previous call on this context; the first
 * call stores u and returns r = +inf.  Synchronises stream.
 */
int rmrt_residual(rmrt_ctx* ctx, double* r, void* stream);

/* Number of steps taken since init (the AA pattern's parity is its low bit). */
int rmrt_steps_taken(const rmrt_ctx* ctx, long long* steps);

/*
 * Checkpoints of a context's state: a header (lattice, equation, storage,
 * pattern, sizes, step count), the stored populations of the current state in
 * their stored layout, and the library-held fields the next steps read (the
 * previous step's phi of the C = 0 form; the previous-step source of the
 * gamma = 0 form with source fields).  A context restored from a checkpoint
 * continues bit for bit as the saved context would have (same kernels, same
 * parity).  Caller-owned inputs (solid mask, source fields) are not part of
 * the checkpoint.
 *   rmrt_checkpoint_bytes   size of the checkpoint of ctx (host only)
 *   rmrt_checkpoint_save    writes it to dst (device or host memory of that
 *                           size); synchronises stream
 *   rmrt_checkpoint_restore reads it from src into ctx, which must have the
 *                           same lattice, equation, storage, pattern, size and
 *                           c_zero, and the same previous-step source field
 *                           (attached, or not); sets the step count and restarts
 *                           the residual; synchronises stream.  RMRT_EINVAL for
 *                           a mismatch, a foreign buffer or a domain of a batch.
 */
int rmrt_checkpoint_bytes(const rmrt_ctx* ctx, size_t* bytes);
int rmrt_checkpoint_save(rmrt_ctx* ctx, void* dst, void* stream);
int rmrt_checkpoint_restore(rmrt_ctx* ctx, const void* src, void* stream);

/*
 * Launch shape of rmrt_step.  flags = 0: one workgroup per 256-node tile
 * (hardware scheduling); blocks_per_cu > 0 then caps the resident workgroups
 * per compute unit through dynamic LDS (0 = no cap).  flags & RMRT_LAUNCH_
 * PERSISTENT: a persistent grid of blocks_per_cu workgroups per CU walks the
 * tiles, contiguously per XCD when flags & RMRT_LAUNCH_XCD_ORDER.
 * Default (measured on MI355X): one workgroup per tile with buffer addressing
 * and the alternating tile order (RMRT_LAUNCH_BUFFER_OFFSETS |
 * RMRT_LAUNCH_ALTERNATE_ORDER); a cap of 4 for rD3Q19 FP32 and for rD3Q27
 * FP32 with walls, a solid mask or a source / force, of 3 for the periodic,
 * unforced rD3Q27 FP32 step, for rD3Q19 and rD3Q27 FP64 and for rD3Q7 FP64;
 * XCD order for rD2Q9, rD2Q5 and rD3Q7 FP32/FP16; RMRT_LAUNCH_XCD_CHUNKS for
 * the other cases whose rows (n[0] x the storage element size) are not a
 * whole number of 128-byte cache lines.  Invalidates the context's cached
 * graphs.
 */
#define RMRT_LAUNCH_XCD_ORDER 1
#define RMRT_LAUNCH_PERSISTENT 2
#define RMRT_LAUNCH_WIDE_TILES 4   /* 512-node tiles, two nodes per thread read before either collides */
/* Buffer addressing of the population streams: the stream start is a scalar
 * 32-bit byte offset and the node a per-lane one, which saves the per-access
 * 64-bit address arithmetic (waves with a bounced link select full 32-bit
 * per-lane offsets instead).  Honoured for population buffers below 4 GiB; a
 * no-op otherwise.  Results are bitwise those of the 64-bit form.  Part of
 * every default launch; batches use it whenever every domain qualifies. */
#define RMRT_LAUNCH_BUFFER_OFFSETS 8
/* Alternating tile order: odd steps walk the tiles backwards, so that every
 * step starts on the nodes the previous step finished with, whose data the
 * memory-side cache (MALL) and the L2 still hold.  Results are bitwise those
 * of the forward order (nodes of one step are independent).  Part of every
 * default launch; batches and rmrt_tune always use it. */
#define RMRT_LAUNCH_ALTERNATE_ORDER 16
/* XCD chunks (one workgroup per tile; ignored by persistent grids; applied
 * to the odd AA steps and to AB steps, the ones that access neighbours'
 * slots): runs of 16 consecutive tiles go to one XCD, the eight XCDs' runs
 * interleaved, so that cache lines straddling two tiles are mostly written
 * through one L2 (neighbour offsets straddle tiles whenever a row is not a
 * whole number of cache lines).  Results are bitwise those of the plain
 * order. */
#define RMRT_LAUNCH_XCD_CHUNKS 32
int rmrt_set_launch(rmrt_ctx* ctx, int blocks_per_cu, int flags);
int rmrt_get_launch(const rmrt_ctx* ctx, int* blocks_per_cu, int* flags);

/*
 * Time rmrt_step over `steps` steps for one workgroup per tile with the
 * residency cap blocks_per_cu in {0 (none), 2, 3, 4, 5, 6, 8}, with 256- and
 * 512-node tiles, with and without RMRT_LAUNCH_BUFFER_OFFSETS where it
 * applies and RMRT_LAUNCH_XCD_CHUNKS where rows straddle cache lines (HIP
 * events on stream), keep the fastest and return its cap
 * in *blocks_per_cu (may be NULL; rmrt_get_launch gives the flags).  The
 * timing runs advance the state.
 */
int rmrt_tune(rmrt_ctx* ctx, int steps, void* stream, int* blocks_per_cu);

/* Release the context (does not free the caller's buffers).  Waits for the
 * device's outstanding work first, since it may still use the context. */
int rmrt_free(rmrt_ctx* ctx);

/*
 * Linear stability preflight of a parameter set (a check before a long run,
 * not part of the method): the collide-and-stream step of eq. 2-2-3 with
 * p's lattice, spacings, rates and variants, in FP64 on a periodic 16 x 16
 * (x 16) domain without walls, solids, force or source, evolves a zero-mean
 * pseudo-random perturbation (amplitude 1e-7 on every stored population) of
 * the uniform state rho = p->rho0 (phi0 for the NCDE), u = u0 (NSE; double[3]
 * host array, NULL for rest), renormalised to its first size after each of 8
 * legs of about steps / 8 (even) steps: a power iteration of the linearised
 * step.  *growth = the mean growth of the perturbation's 2-norm per step over
 * the last 4 legs; it tends to the largest amplification factor |lambda(k)|
 * of the linearised step over the domain's wave vectors (von Neumann
 * analysis), so > 1 flags a parameter set whose small disturbances grow.
 * INFINITY when the perturbation overflows within a leg.  steps in [16, 1e6]
 * (a few thousand resolve growth rates of 1e-3 per step); RMRT_EINVAL for NULL
 * pointers or steps out of range, and every error rmrt_derive returns for p.
 * Allocates and frees its own device memory; synchronous on stream.
 */
int rmrt_preflight(const rmrt_params* p, const double* u0, int steps, double* growth, void* stream);

/*
 * Index-checked build (librmrt_checked.so, the library compiled with
 * RMRT_CHECKED=1 in its host code and FP64 kernels; not for production runs):
 * every neighbour node index the kernels compute (streaming in the odd AA and
 * the AB steps, swapped-layout reads of the companion kernels, solid-mask and
 * velocity-gradient neighbours) is tested against the domain's node count;
 * an index outside it is counted in a per-context device counter and
 * replaced by the node's own index, so that no access leaves the buffers.
 * rmrt_checked_build returns 1 in that build and 0 in the production one.
 * rmrt_checked_violations copies the counter to *count (synchronous on
 * stream).  rmrt_checked_set_limit lowers the bound the checks use to limit
 * (in [1, N]) and clears the counter: a test of the checks themselves, whose
 * nodes at and above limit then count as out of range while every access
 * stays inside the buffers.  Both return RMRT_EUNSUPPORTED in the production
 * build and RMRT_EINVAL for NULL pointers or a limit out of range.
 */
int rmrt_checked_build(void);
int rmrt_checked_violations(rmrt_ctx* ctx, unsigned* count, void* stream);
int rmrt_checked_set_limit(rmrt_ctx* ctx, unsigned limit, void* stream);

/*
 * Batched persistent stepping of nd independent domains that share lattice,
 * equation, storage, pattern and forcing on/off, but not sizes, spacings,
 * viscosities or walls.  One persistent kernel per step processes a static
 * list of (domain, node-range) tiles; rmrt_batch_step replays a HIP graph of
 * nsteps such launches.
 *   params  array of nd parameter sets
 *   f0, f1  arrays of nd device population buffers (f1 NULL for RMRT_AA)
 *   solid   array of nd device masks or NULL (the array or any entry)
 * Populations are initialised to rest (rho = rho0, u = 0 plus -dt F / 2).
 */
int rmrt_batch_create(rmrt_batch** out, int nd, const rmrt_params* params, void* const* f0,
                      void* const* f1, const uint8_t* const* solid, void* stream);

/* Borrow the context of domain d (for rmrt_set_fields/moments/reduce/residual/populations;
 * rmrt_step on it returns RMRT_EINVAL).  Owned by the batch. */
int rmrt_batch_domain(rmrt_batch* b, int d, rmrt_ctx** out);

/*
 * Time every tile configuration of the built-in candidate list over `steps`
 * steps each (HIP events on stream), keep the fastest and return its index in
 * *chosen (may be NULL); then time the domain groups of
 * rmrt_batch_set_group_bytes (none, 128, 192 or 256 MiB) with that
 * configuration and keep the fastest; then, when a group holds a domain whose
 * rows straddle cache lines and the chosen shape is not persistent, time
 * rmrt_batch_set_xcd_chunks modes 1 and 0 and keep the faster.  The timing
 * runs advance the state; call rmrt_set_fields afterwards when the initial
 * state matters.
 */
int rmrt_batch_autotune(rmrt_batch* b, int steps, void* stream, int* chosen);

/*
 * Domain groups: consecutive domains whose population buffers add up to at
 * most `bytes` (a larger domain alone) form a group, and rmrt_batch_step(n)
 * advances each group through its n steps before the next group starts, so
 * that a group that fits in the memory-side cache (MALL, 256 MB) keeps its
 * populations there from step to step.  The domains are independent, so the
 * results are bitwise those of stepping all domains together.  bytes = 0 (the
 * default): one group, one launch per step for the whole batch; otherwise one
 * launch per group and step.  rmrt_batch_get_group_bytes returns the setting
 * and the number of groups (either pointer may be NULL).  RMRT_EINVAL for a
 * NULL batch.  Changing the setting drops the batch's cached graphs.
 */
int rmrt_batch_set_group_bytes(rmrt_batch* b, size_t bytes);
int rmrt_batch_get_group_bytes(const rmrt_batch* b, size_t* bytes, int* ngroups);

/*
 * XCD chunks for batches (see RMRT_LAUNCH_XCD_CHUNKS): mode 1 (the default)
 * launches with them every group that holds a domain whose rows are not a
 * whole number of 128-byte cache lines (n[0] x the storage element size), when
 * the tile shape is one workgroup per tile; mode 0 never.  Results are
 * bitwise the same either way.  rmrt_batch_get_xcd_chunks returns the mode
 * and how many groups qualify (either pointer may be NULL).  RMRT_EINVAL for a
 * NULL batch or another mode.  Changing the mode drops the cached graphs.
 */
int rmrt_batch_set_xcd_chunks(rmrt_batch* b, int mode);
int rmrt_batch_get_xcd_chunks(const rmrt_batch* b, int* mode, int* chunked_groups);

/* Select tile configuration `cfg` (0 .. rmrt_batch_num_configs()-1) explicitly. */
int rmrt_batch_set_config(rmrt_batch* b, int cfg);
int rmrt_batch_num_configs(void);
/*
 * Describe configuration cfg: threads per workgroup, nodes per tile, workgroups
 * per CU, whether the grid is persistent (1: cus * blocks_per_cu workgroups
 * walk the tile list in XCD-contiguous order; 0: one workgroup per tile with
 * residency capped at blocks_per_cu per CU, 0 = no cap) and nodes per thread
 * per pass (2: each thread reads two nodes before colliding either).  Any
 * output pointer may be NULL.
 */
int rmrt_batch_config_info(int cfg, int* threads, int* tile_nodes, int* blocks_per_cu, int* persistent,
                           int* nodes_per_thread);

/* Advance every domain nsteps steps (graph replay of persistent launches). */
int rmrt_batch_step(rmrt_batch* b, int nsteps, void* stream);

/* rmrt_step_prepare for a batch: capture, instantiate and upload the graphs
 * of rmrt_batch_step(b, nsteps) for the current tile configuration and
 * domain groups, without running them. */
int rmrt_batch_step_prepare(rmrt_batch* b, int nsteps, void* stream);

/*
 * rmrt_residual for every domain of the batch with one host synchronisation:
 * r[d] = ||u^n - u^prev||_2 / ||u^n||_2 (phi for the NCDE) against the
 * previous call (first call: +inf).  r holds nd doubles (host).  Returns
 * RMRT_ENONFINITE (r[d] = NaN) when a domain's sums are not finite.
 */
int rmrt_batch_residual(rmrt_batch* b, double* r, void* stream);

/* Release the batch and its domain contexts (not the caller's buffers); waits
 * for the device's outstanding work first. */
int rmrt_batch_free(rmrt_batch* b);

/* ===========================================================================
 * Warm-start surrogate (not part of the paper's method): a network of 3x3
 * dilated convolutions that predicts a steady channel flow from its geometry,
 * used to initialise the populations through rmrt_set_fields with
 * with_fne = 1 (Sec. IV eq. fne).  All kernels are hand-written for gfx950;
 * convolutions are implicit GEMMs on MFMA (bf16 inputs, fp32 accumulation).
 *
 * Layouts: activations (B, H, W, C) channels-last with C = 16 or 32; weights
 * (Cout, 3, 3, Cin); bf16 tensors are raw 16-bit bfloat16.  Tap (ky, kx)
 * reads (h + (ky - 1) dil, w + (kx - 1) dil), zero outside the image.
 * Every pointer is caller-owned device memory; every call is asynchronous on
 * stream.
 * ======================================================================== */

/* epilogues of rmrt_nn_conv_forward */
#define RMRT_NN_EPI_NONE 0       /* a = y                                   */
#define RMRT_NN_EPI_SILU 1       /* a = silu(y)                             */
#define RMRT_NN_EPI_SILU_GRAD 2  /* a = y * silu'(aux)  (backward pass)     */

/*
 * y = bias + conv3x3(x, w, dil); y_pre (fp32, may be NULL) receives y and
 * a_out (bf16, may be NULL) the epilogue applied to y.  bias may be NULL.
 * Cin, Cout in {16, 32}.
 */
int rmrt_nn_conv_forward(const void* x, const void* w, const float* bias, float* y_pre, void* a_out,
                         const float* aux, int B, int H, int W, int Cin, int Cout, int dil, int epilogue,
                         void* stream);

/* wt[ci][ky][kx][co] = w[co][2-ky][2-kx][ci]: backward-data is rmrt_nn_conv_forward with wt. */
int rmrt_nn_flip_weights(const void* w, void* wt, int Cout, int Cin, void* stream);

/* Scratch floats needed by rmrt_nn_conv_backward_weight. Host only. */
size_t rmrt_nn_wgrad_scratch_floats(int B, int H, int W, int Cin, int Cout);

/*
 * dw[co][ky][kx][ci] = sum_p dy[p][co] x[p + tap][ci] and db[co] = sum_p dy[p][co]
 * (db may be NULL); x, dy bf16, dw, db fp32; deterministic (fixed-order sums).
 */
int rmrt_nn_conv_backward_weight(const void* x, const void* dy, int B, int H, int W, int Cin, int Cout, int dil,
                                 float* dw, float* db, float* scratch, size_t scratch_floats, void* stream);

/*
 * Weighted MSE over the first C channels of out (fp32, row stride out_stride):
 * loss = sum_p weight[p] sum_c (out - target)^2 / sum_p weight[p] into *loss
 * (device double); dout (bf16, stride out_stride) = dloss/dout, zero in the
 * padding channels.  target is (P, C) fp32; scratch holds 1024 doubles and
 * inv_den one float.
 */
int rmrt_nn_masked_mse(const float* out, int out_stride, const float* target, const float* weight, long P, int C,
                       void* dout, double* scratch, float* inv_den, double* loss, void* stream);

/* Adam step t >= 1 (bias-corrected) on n fp32 parameters; w_bf16 (may be NULL) receives a bf16 copy. */
int rmrt_nn_adam(float* w, void* w_bf16, const float* g, float* m, float* v, long n, float lr, float b1, float b2,
                 float eps, int t, void* stream);

/* dst (bf16) = round-to-nearest-even(src). */
int rmrt_nn_to_bf16(const float* src, void* dst, long n, void* stream);

/*
 * Network input on the k-coarsened grid of B channels of nx x ny nodes (walls
 * at the y faces, spacing dy): channel 0 = solid fraction of each k x k block,
 * 1 = Poiseuille prior 4 y (H - y) / H^2 at the block centre, 2 = Re / re_scale,
 * 3 = solid fraction of the block's columns over the full height, 4 = solid
 * fraction of the whole channel, the rest 0.  solid is (B, ny, nx) uint8, re
 * is B floats, x0 is (B, ny/k, nx/k, channels >= 5) bf16, scratch holds
 * B (nx + 1) floats.
 */
int rmrt_nn_features(const uint8_t* solid, const float* re, int B, int nx, int ny, int k, float dy, float re_scale,
                     void* x0, int channels, float* scratch, void* stream);

/*
 * Training targets from steady fields (rho: B x N, u: B x 2 x N doubles, the
 * layout of rmrt_moments): fluid means over each block of u / Ut - prior(y),
 * v / Ut and (rho - 1) rho_scale into tgt (B, ny/k, nx/k, 3) fp32, and the
 * fluid fraction of the block into wgt.
 */
int rmrt_nn_targets(const double* rho, const double* u, const uint8_t* solid, int B, int nx, int ny, int k, float dy,
                    float Ut, float rho_scale, float* tgt, float* wgt, void* stream);

/*
 * Initial fields from the network output (B, ny/k, nx/k, out_stride) fp32:
 * bilinear upsampling to the nodes, then u = Ut (prior + o0), v = Ut o1,
 * rho = 1 + o2 / rho_scale, u = 0 in solid nodes (solid may be NULL).
 */
int rmrt_nn_warm_fields(const float* out, int out_stride, int B, int nx, int ny, int k, float dy, float Ut,
                        float rho_scale, const uint8_t* solid, double* rho, double* u, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RMRT_H */
