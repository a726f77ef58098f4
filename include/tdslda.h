/*
 * tdslda.h - C ABI of libtdslda, the MI355X (gfx950) implementation of the
 * time-dependent superfluid local density approximation (TDSLDA) step of the
 * W-SLDA Toolkit paper (arXiv 2602.08982).
 *
 * One step applies the lattice BdG Hamiltonian of the spin-symmetric reduced
 * problem (Sec. 2.3, Eq. HpsiEpsi, with the A_sigma = 1 single-particle
 * Hamiltonian of Eq. h_sigma_A1) to every quasiparticle state (u_n, v_n),
 * with the kinetic term done spectrally (Sec. 3.1, Eq. derivative-spectral)
 * and the mean field U(r) and pairing field Delta(r) applied pointwise;
 * advances all states with the Adams-Bashforth-Moulton predictor-corrector of
 * Sec. 3.3 (Alg. AB4AM5, Eqs. AB3-AM5) on the shifted equation of motion
 * (Eq. ABM-f); and reduces over states to rebuild the densities
 * (Eqs. nab3D-jab3D) that feed the next evaluation's mean fields.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Units hbar = m = k_B = 1 (Sec. 2.1).
 *  - Lattice (Sec. 3.1): periodic, N_x x N_y x N_z sites, even sizes, spacing
 *    dx, dy, dz; flat site index ixyz = (ix*N_y + iy)*N_z + iz (z fastest);
 *    M = N_x N_y N_z.  Physical coordinates x = (ix - N_x/2) dx (centred).
 *    Quasi-1D mode (Sec. 3.1, quasi-1D item): states live on the z axis only
 *    (M = N_z), every state carries its transverse momentum squared
 *    k_perp^2, and the transverse box is L_x x L_y.
 *    Quasi-2D mode (Sec. 3.1, quasi-2D item): states live on the x-y lattice
 *    (M = N_x N_y, flat index ix*N_y + iy, normalised on the x-y lattice),
 *    every state carries its plane-wave momentum squared k_z^2 (one of the
 *    N_z/2 + 1 distinct |k_z| = 2 pi m / L_z, L_z = N_z dz) and a
 *    multiplicity (the two signs of k_z share one problem); densities carry
 *    1/L_z and tau the k_z^2 term.  A = 1 functional only.
 *  - A state is (u_n, v_n) = (u_{n,a}, v_{n,b}); host arrays of states are
 *    double precision, layout [n][2][M][2] (state, component u|v, site,
 *    re|im).  States are normalised as int (|u|^2 + |v|^2) dV = 1.
 *  - Only the E_n > 0 half of the spectrum is evolved (spin-symmetric
 *    reduction, Sec. 2.3); weights f(E_n), f(-E_n) are frozen (Sec. 2.5).
 *  - Host pointers are caller-owned and only read / written during the call.
 *    Device pointers passed in are borrowed: the caller keeps them alive and
 *    orders them on the context's stream.  The context owns everything it
 *    allocates and frees it in tdslda_destroy.
 *  - Every call returns a tdslda_status; on failure tdslda_last_error() gives
 *    a context-owned message valid until the next call on that context.
 *    No call throws across the ABI.  A context is not thread-safe; use one
 *    context per stream.
 */
#ifndef TDSLDA_H
#define TDSLDA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TDSLDA_OK = 0,
  TDSLDA_EINVAL = -1,    /* bad argument, unsupported shape or option */
  TDSLDA_ENOMEM = -2,    /* device allocation failed */
  TDSLDA_EDEVICE = -3,   /* HIP runtime error */
  TDSLDA_EORDER = -4,    /* call out of order (e.g. abm_step before load) */
  TDSLDA_EUNSTABLE = -5  /* conservation or NaN check failed (Sec. 4.5.1) */
} tdslda_status;

enum { TDSLDA_MODE_3D = 3, TDSLDA_MODE_Q1D = 1, TDSLDA_MODE_Q2D = 2 };
enum { TDSLDA_FUNC_SLDA = 1, TDSLDA_FUNC_BDG = 2, TDSLDA_FUNC_ASLDA = 3 };
enum { TDSLDA_FP64 = 0, TDSLDA_FP32_MIXED = 1 };
enum { TDSLDA_AB3AM4 = 34, TDSLDA_AB4AM5 = 45, TDSLDA_AB5AM5 = 55 };

typedef struct tdslda_ctx tdslda_ctx;

typedef struct {
  int mode;             /* TDSLDA_MODE_3D, TDSLDA_MODE_Q1D or TDSLDA_MODE_Q2D */
  int nx, ny, nz;       /* 3D: lattice sizes; Q1D: nx = ny = 1, nz = N_z; Q2D: the
                           x-y lattice nx, ny and nz = N_z plane waves along z */
  double dx, dy, dz;    /* spacings (Q1D: dz only; Q2D: dz sets L_z = nz dz) */
  double lx_perp, ly_perp; /* Q1D: transverse box L_x, L_y (densities carry 1/(L_x L_y)) */
} tdslda_lattice;

typedef struct {
  int functional;       /* TDSLDA_FUNC_SLDA (Sec. 2.4, ASLDA at p=0) or TDSLDA_FUNC_BDG (Eq. HBdG) */
  double A, B, C;       /* SLDA constants.  A = 1: Eq. h_sigma_A1.  A != 1: the general
                           functional of Eq. h_sigma (alpha = A, current potential
                           (1 - A) j / rho, rebuilt with j at every field build) */
  double inv_g_bdg;     /* BdG: 1/(4 pi a_s) */
  double ec_reg;        /* cut-off energy E_c of the regulator Lambda_c (Eq. Creg) */
  double mu;            /* chemical potential, fixed during TD (ASLDA: mu_a) */
  double temperature;   /* T of the frozen weights f(E) = 1/(exp(E/T)+1); 0 = step */
  double mu_b;          /* ASLDA: chemical potential of spin b (else unused) */
} tdslda_functional;
/* TDSLDA_FUNC_ASLDA (Sec. 2.4, ASLDA item; quasi-1D and full-3D contexts): the
 * spin-imbalanced functional with A_a(p) = A(p), A_b(p) = A(-p), B(p) and
 * C = -11.11 of the local polarisation p = (rho_a - rho_b) / rho_+.  Both
 * branches of Eq. HpsiEpsi are evolved (load states of either sign of E; no
 * E > 0 halving), the u row carries h_a - mu_a and the v row -h_b^* + mu_b,
 * each h of Eq. h_sigma with its own alpha_s = A_s, current potential
 * (1 - A_s) j_s / rho_s and V_s = dE/drho_s (the p-dependence of A_s and B
 * included), densities of Eqs. na3D-jb3D (quasi-1D: with 1/(L_x L_y)).  The fields
 * A, B of this struct are not used.  Linear mode, friction and the
 * general-operator fields are refused; tdslda_densities_spin gives the
 * densities.  The regulator frozen by tdslda_set_external uses the spin
 * averages A_+ = A(0), mu_+ = (mu_a + mu_b) / 2 (Eq. Creg). */

typedef struct {
  int precision;        /* TDSLDA_FP64 or TDSLDA_FP32_MIXED (states, transforms and H.psi
                           in FP32; densities, norms, <H>_n, energy in FP64) */
  int integrator;       /* TDSLDA_AB3AM4, TDSLDA_AB4AM5 (default), TDSLDA_AB5AM5 */
  double dt;            /* time step (internal units) */
  int selfstart;        /* 0: states stationary (every history slot = f(phi_0));
                           1: Taylor predictor-corrector start-up (Eq. Taylor-exp) */
  int taylor_order;     /* r of the Taylor start-up (0 selects 5) */
  double tol_N, tol_E;  /* relative tolerances of the conservation check done by
                           tdslda_check (<= 0 disables that check) */
  void* hip_stream;     /* borrowed hipStream_t (NULL = the null stream) */
} tdslda_run;

/* Create a context for up to `capacity` evolved states and allocate its
 * device buffers: (history depth + 1) state buffers plus one intermediate
 * buffer (the x-derivative of every state), per-state scalars and the FP64
 * fields.  Supported shapes: cubic N^3 with N in {4,6,8,12,16,24,32,48},
 * 8x8x16 (3D); N_z in {16,64,256} (Q1D: N_z = A^2 with A lanes per state);
 * N_x x N_y in {8x8, 12x12, 16x16, 24x16, 32x32, 48x48, 64x64} (Q2D: a state
 * per workgroup, its 2D Laplacian in LDS; no intermediate buffer).  The
 * quasi-1D evaluations use the intermediate buffer only in the start-up.
 * Full-3D contexts hold at most 65535 states.  Errors: EINVAL (including an
 * unsupported shape, a 3D capacity above 65535, and A != 1 in Q2D),
 * ENOMEM. */
tdslda_status tdslda_create(const tdslda_lattice* lat, const tdslda_functional* fun,
                            const tdslda_run* run, int64_t capacity, tdslda_ctx** out);
tdslda_status tdslda_destroy(tdslda_ctx* ctx);
const char* tdslda_last_error(const tdslda_ctx* ctx);

/* Bytes of device memory tdslda_create would allocate for `nstates`
 * (the td-memory estimate of Sec. 4.5.3, for this library's buffers). */
tdslda_status tdslda_memory_plan(const tdslda_lattice* lat, const tdslda_run* run,
                                 int64_t nstates, int64_t* bytes_out);

/* External fields (Sec. 2.2, Eq. E_tot), switched on from now on:
 * V_ext[M] (host, FP64) and the external pairing potential
 * Delta_ext[M][2] (host, FP64 re|im; NULL = 0).  H then carries U + V_ext -
 * mu on the diagonal and Delta + Delta_ext off the diagonal (Eq. HpsiEpsi
 * and its time-dependent form), in linear mode too; Delta itself stays
 * -g_eff nu, and tdslda_energy adds E_pair.ext = -int (Delta_ext nu^* +
 * c.c.).  With a non-zero Delta_ext the particle number is not conserved
 * and tdslda_check checks E - mu N only.  If freeze_regulator != 0 the
 * regulator Lambda_c(r) of Eq. Creg is (re)computed from V_ext with V_+ =
 * V_ext and then kept frozen (the regulator is never refreshed during TD).
 * Errors: EINVAL (vext NULL, non-finite Delta_ext, E_c below the local band
 * bottom). */
tdslda_status tdslda_set_external(tdslda_ctx* ctx, const double* vext, const double* dext_reim,
                                  int freeze_regulator);
/* Set the frozen regulator Lambda_c[M] directly (host, FP64). */
tdslda_status tdslda_set_regulator(tdslda_ctx* ctx, const double* lam);

/* Load n <= capacity states (host, [n][2][M][2] FP64, copied and rounded to
 * the context precision) with their static quasiparticle energies E[n] (the
 * frozen weights f(E), f(-E) are computed from them) and, in Q1D mode,
 * kperp2[n], in Q2D mode k_z^2 in the same array (else NULL).  Every
 * multiplicity is reset to 1.  Resets the integrator. */
tdslda_status tdslda_load_states(tdslda_ctx* ctx, int64_t n, const double* uv, const double* E,
                                 const double* kperp2);
/* Same from a device array of the context precision ([n][2][M] complex of
 * double or float, interleaved re/im), copied. */
tdslda_status tdslda_load_states_device(tdslda_ctx* ctx, int64_t n, const void* uv_dev,
                                        const double* E, const double* kperp2);

/* Multiplicity of each loaded state (host FP64 [n], n = the loaded count,
 * each > 0): the weights become mult f(E), mult f(-E), so that one evolved
 * state stands for mult equal problems (Q2D: 2 for the classes 0 < |k_z| <
 * the Nyquist momentum, whose +k_z and -k_z problems coincide; Sec. 3.1,
 * quasi-2D item).  Between a load and the first step only; the fields are
 * rebuilt.  Errors: EINVAL (count, values), EORDER (nothing loaded, or
 * the integrator already started). */
tdslda_status tdslda_set_multiplicity(tdslda_ctx* ctx, int64_t n, const double* mult);

/* Uniform-system start (Sec. 4.5.1 "uniform-system solution"): n plane-wave
 * eigenstates of the uniform H with constant U = u0 and Delta = delta0
 * (real, > 0) at momenta k = 2 pi m / L with integer triples kidx[n][3]
 * (grid indices 0..N-1 of Sec. 3.1), generated on the device:
 * u = sqrt((1 + xi/E)/2), v = sqrt((1 - xi/E)/2), xi = k^2/2 + u0 - mu,
 * times exp(i k.r)/sqrt(V).  E_n of each state sets its frozen weights.
 * Q2D: kidx[n] = (l_x, l_y, m) with m in [0, nz/2] the |k_z| class
 * (k_z = 2 pi m / L_z enters xi), the x-y plane wave normalised on the x-y
 * lattice, and the multiplicity of the class (1 for m = 0 and m = nz/2,
 * else 2) set with k_z^2.  ASLDA (3D): both branches of every listed
 * momentum, 2n states (capacity >= 2n): with constant fields the
 * imbalanced problem is the balanced one at the spin-averaged
 * xi = k^2/2 + u0 - (mu_a + mu_b)/2, shifted by -(mu_a - mu_b)/2, so state
 * 2i is (u, v) above at E = -(mu_a - mu_b)/2 + e and state 2i + 1 its
 * partner (-v, u) at -(mu_a - mu_b)/2 - e, e = sqrt(xi^2 + delta0^2).
 * Errors: EINVAL (Q1D context, n or an index out of range, delta0 <= 0). */
tdslda_status tdslda_init_plane_waves(tdslda_ctx* ctx, int64_t n, const int32_t* kidx,
                                      double u0, double delta0);
/* Vortex imprint on every loaded state (a phase e^{i theta} on Delta; Delta
 * is derived from the states in TD, so the phase goes onto the states as
 * the local gauge rotation of both fermion fields by theta/2): u_n <- e^{i theta/2} u_n, v_n <- e^{-i theta/2} v_n, which
 * multiplies nu and Delta by e^{i theta}, keeps rho and the orthonormality
 * of the states, and commutes with the partner map (u, v) -> (v^*, -u^*) of
 * the spin-symmetric reduction (Sec. 2.3), so the evolved E > 0 states keep
 * standing for a complete set.  theta = sum_j q_j atan2(y - y_j, x - x_j)
 * (straight lines along z, centred coordinates).  xyq: [nv][3] host array
 * of (x_j, y_j, q_j).  3D and Q2D. */
tdslda_status tdslda_imprint_vortices(tdslda_ctx* ctx, int nv, const double* xyq);

/* Linear-mode potentials of the general single-particle Hamiltonian
 * (Sec. 2.3, Eq. h_sigma), host FP64, for a context with frozen fields
 * (tdslda_set_fields first): alpha[M] (inverse effective mass, > 0) and the
 * current potential avec (3D: [3][M], components x, y, z; quasi-1D: [M], the
 * z component; the transverse ones vanish).  H then applies
 *   h = -1/2 div(alpha grad) + U + V_ext - mu - (i/2) {A, grad}
 * (quasi-1D: + 1/2 alpha k_perp^2) with the kinetic part in the symmetrised
 * form of Eq. kinop-alpha (1/2 [D2(alpha x) + alpha D2 x - x D2 alpha] per
 * axis, D2 of Eq. D2) and the current part A_d D1_d x + D1_d(A_d x) (Eqs.
 * Ad_dx, d_dxA; D1 with the Nyquist mode zeroed), 7 transforms per
 * component and axis; -h^* on v.  A NULL array keeps the functional's value
 * (alpha = A, A = 0); both NULL return to the functional's potentials.
 * tdslda_set_fields(NULL, NULL) also resets them.  Errors: EINVAL
 * (non-finite values, alpha <= 0), EORDER (fields not frozen). */
tdslda_status tdslda_set_current_fields(tdslda_ctx* ctx, const double* alpha, const double* avec);

/* Freeze the mean fields (linear mode): U[M] and Delta[M][2] (host FP64) are
 * used by every later H application and never rebuilt.  Pass NULLs to go
 * back to self-consistent fields. */
tdslda_status tdslda_set_fields(tdslda_ctx* ctx, const double* U, const double* delta_reim);

/* Densities of the current states (Eqs. nab3D-jab3D, per spin component),
 * FP64, host outputs (any may be NULL): rho[M], tau[M], nu[M][2], j[3][M].
 * tau gives the Nyquist mode its full weight (pi/dx)^2 with the Nyquist
 * momentum taken symmetrically; j uses the first derivative with the Nyquist
 * mode zeroed (Sec. 3.1).  Also refreshes the mean fields from rho, nu
 * unless they are frozen. */
tdslda_status tdslda_densities(tdslda_ctx* ctx, double* rho, double* tau, double* nu_reim, double* j);
/* Spin-resolved densities of an ASLDA context (Eqs. na3D-jb3D), FP64 host
 * outputs (any may be NULL): rho[2][M], tau[2][M] (spin a then b), nu[M][2],
 * j[2][3][M] (x, y, z components of j_a, then j_b; quasi-1D: z only, x and y
 * zero).  Also refreshes the mean fields.
 * Errors: EINVAL (not an ASLDA context), EORDER (nothing loaded). */
tdslda_status tdslda_densities_spin(tdslda_ctx* ctx, double* rho, double* tau, double* nu_reim, double* j);
/* Current mean fields (host FP64 out, any may be NULL): U[M], Delta[M][2]
 * (ASLDA: U[2][M], V_a then V_b). */
tdslda_status tdslda_get_fields(tdslda_ctx* ctx, double* U, double* delta_reim);

/* H psi with the current fields, unshifted and unnormalised, for n states of
 * device arrays in the context precision (layout as the loaded states).
 * n <= capacity; in and out must not overlap.  Q1D (Q2D): kperp2 (k_z^2) of
 * the loaded state with the same index is used. */
tdslda_status tdslda_apply_hbdg(tdslda_ctx* ctx, const void* in_dev, void* out_dev, int64_t n);

/* Quantum friction (Sec. 5.2, correcting the initial state by a
 * time-dependent approach; Eqs. cooling_alpha, Deltadiss2): from the next
 * field build on, the evolution adds the dissipative fields
 *   U_diss     = -(alpha / rho0) div j,
 *   Delta_diss = Delta [beta sin(theta_nu - theta_B') + i gamma (N - N_req) / N_req],
 * theta_nu = arg nu, theta_B' = arg B', B' = -1/2 sum_n (f_v - f_u)
 * [u lap v^* + v^* lap u] on the normalised states, N = int rho_+ d^3r.
 * 3D: lap the full Laplacian (Eq. D2), div j = sum_d D1_d j_d (D1 with the
 * Nyquist mode zeroed, as j); one line pass per axis for j and for B' over
 * the states, then line passes over the current field.  Quasi-1D: lap =
 * D2z - k_perp^2 and div j = D1z j_z, with 1/(L_x L_y); one pass over the
 * states (four-step DFTs).  The gamma term is off when N_req <= 0; all of
 * alpha, beta and the gamma term zero switch friction off.  Not with the
 * general (A != 1) operator, not in Q2D; not stored by tdslda_save.
 * Errors: EINVAL (general operator, Q2D, non-finite parameters,
 * rho0 <= 0), ENOMEM. */
tdslda_status tdslda_set_friction(tdslda_ctx* ctx, double alpha, double beta, double gamma, double rho0,
                                  double N_req);

/* Advance the loaded states by nsteps steps of the selected ABM integrator.
 * The first call after a load runs the start-up (selfstart), which is not
 * counted in nsteps.  Errors: EORDER before any load. */
tdslda_status tdslda_abm_step(tdslda_ctx* ctx, int64_t nsteps);

/* The same advance as tdslda_abm_step, recorded once as a HIP graph on the
 * context's stream (a private stream, created once per context, when the
 * context uses the null stream) and submitted as one launch: every kernel
 * boundary of the recording is a grid-wide synchronisation point (density
 * reductions included).  The call returns after the launch has completed;
 * the executed graph is released at the next call or by tdslda_destroy.  Requires
 * a started integrator (one tdslda_abm_step call, nsteps >= 0, after the
 * load) and profiling off.  graph_ms (may be NULL) = {record + instantiate
 * time, launch-to-completion time} in milliseconds.  If recording or
 * instantiation fails, nothing has run and the context is left as before
 * the call; if the launch itself fails, the context drops its states (a
 * later call needs a new load, EORDER until then).
 * Errors: EORDER before the start-up or with profiling on; EDEVICE. */
tdslda_status tdslda_abm_graph(tdslda_ctx* ctx, int64_t nsteps, double graph_ms[2]);

/* Launch-shape tuner: times each candidate workgroup size of every tunable
 * kernel class on the loaded states and keeps the fastest for the rest of
 * the context's life.  Quasi-1D kernel sets tune 4 classes (density pass,
 * z-derivative pass, fused H.psi/integrator passes (timed as one step's
 * corrector and full pass), pointwise pass) over
 * 64/128/256 threads; full-3D sets have fixed shapes (nclasses = 0).  Only
 * scratch buffers are written.  choice[4], ms[4] (host, may be NULL): chosen
 * workgroup size and its median time per class.  Errors: EORDER before a load. */
tdslda_status tdslda_autotune(tdslda_ctx* ctx, int* nclasses, int32_t choice[4], double ms[4]);

/* Static states of the batched quasi-1D problems (Sec. 3.1, quasi-1D item;
 * Sec. 2.3, Eq. HpsiEpsi): for each of nprob transverse momenta kperp2[p]
 * (host) the real 2N_z x 2N_z BdG matrix with
 *   h = -1/2 D2 + hfield(z) + kperp2[p]/2   (D2 of Eq. D2 along z, Nyquist kept)
 * and the real pairing field delta(z) (both host [N_z]; hfield includes
 * U + V - mu) is diagonalised on the device (rocSOLVER, batched) and the
 * eigenpairs with 0 < E < ecut are kept, normalised to int |phi|^2 dz = 1.
 * tdslda_q1d_count: per-problem counts (host int32[nprob]) and their sum,
 * eigenvalues only.  tdslda_q1d_load_static: loads the kept states of all
 * problems, problem by problem in ascending E, as the context's states with
 * their E (weights) and kperp2, like tdslda_load_states; the context must be
 * quasi-1D with capacity >= the total.  Errors: EINVAL (mode, sizes,
 * capacity), EDEVICE (eigensolver failure), ENOMEM. */
tdslda_status tdslda_q1d_count(const tdslda_lattice* lat, int nprob, const double* kperp2, const double* hfield,
                               const double* delta, double ecut, int32_t* counts, int64_t* total);
tdslda_status tdslda_q1d_load_static(tdslda_ctx* ctx, int nprob, const double* kperp2, const double* hfield,
                                     const double* delta, double ecut, int64_t* nloaded);
/* The same for spin-imbalanced problems (Sec. 2.3, Eq. HpsiEpsi without the
 * spin symmetry): the upper block carries hfield_a (h_a - mu_a), the lower
 * -(hfield_b) (-(h_b - mu_b)), and both branches are kept, every eigenpair
 * with |E| < ecut (the states an ASLDA context evolves). */
tdslda_status tdslda_q1d_count_spin(const tdslda_lattice* lat, int nprob, const double* kperp2,
                                    const double* hfield_a, const double* hfield_b, const double* delta, double ecut,
                                    int32_t* counts, int64_t* total);
tdslda_status tdslda_q1d_load_static_spin(tdslda_ctx* ctx, int nprob, const double* kperp2, const double* hfield_a,
                                          const double* hfield_b, const double* delta, double ecut,
                                          int64_t* nloaded);

/* Static self-consistent solve, quasi-2D geometry (Sec. 3.2, Alg. MapK;
 * Sec. 3.1 quasi-2D item): an nx x ny periodic x-y lattice (spacings dx, dy)
 * and nz plane-wave momenta along z (spacing dz, L_z = nz dz); the
 * nz/2 + 1 distinct |k_z| are diagonalised once per iteration (real BdG
 * matrices of order 2 nx ny, one batched rocSOLVER call) with multiplicity
 * weights.  T = 0: every E > 0 eigenpair is occupied.  The map K returns the
 * potentials of the SLDA (A = 1) or BdG functional with the regulator
 * Lambda_c(V_+ = V_ext + U_in, mu, ec).  Fixed-N mode when a_mu != 0
 * (Eq. update-mu, with N = int rho_+ d^3r, is the last step of K).
 * Iteration (Sec. 3.2, the two mixing methods):
 *   broyden = 0: linear mixing of (U, Delta) with parameter mix; mu takes
 *     the update-mu output unmixed;
 *   broyden = m > 0: modified Broyden mixing (the variant the paper cites,
 *     Baran et al., Phys. Rev. C 78, 014318) of p = (U, Delta, mu) with the
 *     last m normalised differences of p and of F = K[p] - p, weights 1 and
 *     w0:  a = w0^2 I + dF dF^T,  gamma = a^-1 (dF . F),
 *     p_new = p + mix F - sum_l gamma_l (mix dF_l + dp_l);  m <= 8.
 * Converged when max(|U_out - U_in|_inf, |Delta_out - Delta_in|_inf) /
 * eF_ref < tol and |N - N_req| / N_req < tol.  Delta is real.  All arrays
 * are host FP64 [nx*ny], flat index ix*ny + iy. */
typedef struct {
  int nx, ny, nz;
  double dx, dy, dz;
  double ec;     /* regulator cutoff E_c */
  double mix;    /* linear mixing parameter m_p in (0, 1] */
  double a_mu;   /* step of Eq. update-mu; 0 = fixed mu */
  double N_req;  /* required particle number (fixed-N mode) */
  double tol;    /* residual threshold */
  double eF_ref; /* Fermi energy of the reference uniform system */
  int maxit;
  int broyden;   /* history length of the Broyden mixing (0..8); 0 = linear mixing */
  double w0;     /* Broyden regularisation weight (e.g. 0.01) */
  int q1d;       /* 1: quasi-1D geometry (Sec. 3.1, quasi-1D item; the first stage of releasing
                    symmetry constraints, Sec. 5.2): an nx-site x lattice with ny plane waves
                    along y (spacing dy, L_y = ny dy) and nz along z; the distinct (|k_y|, |k_z|)
                    pairs are diagonalised (order 2 nx) with multiplicities, densities carry
                    1/(L_y L_z) and fields are [nx].  0: the quasi-2D geometry above */
} tdslda_static;

/* One application of K at (U, delta, mu): U_out, delta_out, rho (per spin),
 * nu (any output may be NULL) and N. */
tdslda_status tdslda_static_map(const tdslda_static* s, const tdslda_functional* fun, const double* vext,
                                const double* U, const double* delta, double mu, double* U_out,
                                double* delta_out, double* rho, double* nu, double* N);
/* Iterate from (U, delta, mu) (updated in place: the converged K output, or
 * the last mixed iterate when maxit is reached).  iters, converged and
 * hist[maxit][4] = {r, |N - N_req|/N_req, mu, N} per iteration may be NULL.
 * Errors: EINVAL, ENOMEM, EDEVICE (eigensolver), EUNSTABLE (non-finite
 * residual or undefined regulator). */
tdslda_status tdslda_static_solve(const tdslda_static* s, const tdslda_functional* fun, const double* vext,
                                  double* U, double* delta, double* mu, int* iters, int* converged,
                                  double* hist);

/* Fourier interpolation of a real field between two lattices of one
 * periodic x-y box (Sec. 5.2, refining lattice resolution: a solution on a
 * coarse lattice is interpolated onto the target lattice as its initial
 * guess).  f: host FP64 [nx*ny] (index ix*ny + iy) with spacings dx, dy;
 * out: host FP64 [nx2*ny2] with spacings dx2, dy2; nx dx = nx2 dx2 and
 * ny dy = ny2 dy2.  out = Re 1/(L_x L_y) sum_lm f~_lm exp[i (k_l x + k_m y)]
 * with f~ the lattice Fourier coefficients of f (k grid of Sec. 3.1,
 * Nyquist at -pi/d) and positions measured from the shared box corner, so
 * points shared by the two lattices keep their values.  Direct sums on the
 * device (coefficients, then one thread per target site).  Errors: EINVAL
 * (sizes, odd source sizes, spacings, box mismatch), ENOMEM. */
tdslda_status tdslda_interp2d(int nx, int ny, double dx, double dy, const double* f, int nx2, int ny2, double dx2,
                              double dy2, double* out);

/* Allocation-free variant of tdslda_interp2d, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same operation and result as
 * tdslda_interp2d, but f_dev (FP64 [nx*ny]) and out_dev (FP64 [nx2*ny2])
 * are caller-owned device arrays, the two kernels are queued on hip_stream
 * (a hipStream_t; NULL = the null stream) and the call returns without
 * waiting.  The Fourier coefficients go to a fixed device array of the
 * library (1 MiB per GPU, held until the process ends) instead of a
 * per-call allocation, which limits the source lattice to nx * ny <= 65536;
 * the call performs no hipMalloc, hipFree or other allocation.  Every call
 * on one GPU shares that array: calls that overlap in time on the same GPU
 * (different streams, or threads) race and must be serialised by the
 * caller.  Nothing in the array needs clearing (each call writes every
 * coefficient it reads).  Errors: EINVAL (NULL pointers, sizes, source
 * lattice beyond the limit, spacings, box mismatch), EDEVICE (launch
 * failure, no device). */
tdslda_status tdslda_interp2d_noalloc(int nx, int ny, double dx, double dy, const double* f_dev, int nx2, int ny2,
                                      double dx2, double dy2, double* out_dev, void* hip_stream);

/* Warm-start network of the static workflow (learned initial guess for
 * the fixed-point iteration of Alg. MapK; Sec. 5.2 on initial guesses).
 * A small convolutional network maps the normalised external potential of
 * an H x W x-y lattice (host float [B][H][W]) to normalised (U, Delta) maps
 * ([B][2][H][W]) and a chemical potential ([B]):
 *   h1 = relu(conv3(x)), h2 = relu(conv3(h1)), h3 = relu(conv3(h2)) (C
 *   channels each, 3x3 kernels with periodic padding), maps = 1x1 conv of
 *   h3, mu = mean over sites of h3 . w_mu + b_mu.
 * Loss L = mean((maps - Y)^2) + lam_mu mean((mu - y_mu)^2); Adam (beta1 0.9,
 * beta2 0.999, eps 1e-8) on FP32 master weights.  Flat parameter order
 * W1 b1 W2 b2 W3 b3 Wm bm w_mu b_mu (conv weights [Cout][Cin][3][3]);
 * tdslda_nn_nparams(C) gives the count.  Initial weights are the caller's.
 * All buffers are device-resident and owned by the network object; host
 * arrays are copied.  Errors: EINVAL (sizes, B > batch_max), ENOMEM, EDEVICE. */
typedef struct tdslda_nn tdslda_nn;
int64_t tdslda_nn_nparams(int C);
tdslda_status tdslda_nn_create(int H, int W, int C, int batch_max, const float* theta0, tdslda_nn** out);
tdslda_status tdslda_nn_destroy(tdslda_nn* nn);
tdslda_status tdslda_nn_params(tdslda_nn* nn, float* theta_out, int64_t* count);
/* replaces the weights and resets the Adam moments and step count */
tdslda_status tdslda_nn_set_params(tdslda_nn* nn, const float* theta);
tdslda_status tdslda_nn_forward(tdslda_nn* nn, int B, const float* x, float* maps, float* mu);
tdslda_status tdslda_nn_loss_grad(tdslda_nn* nn, int B, const float* x, const float* Y, const float* y_mu,
                                  float lam_mu, float* loss, float* grad);
/* loss_grad followed by one Adam step with learning rate lr */
tdslda_status tdslda_nn_train_step(tdslda_nn* nn, int B, const float* x, const float* Y, const float* y_mu,
                                   float lam_mu, float lr, float* loss);

/* Energy terms of Sec. 3.2 for the current states, host out[9]:
 * {E_kin, E_pot, E_pair, E_curr, E_pot.ext, E_total, N, E_FG, E_pair.ext}
 * with E_total the sum of the five terms and E_pair.ext, N = int rho_+ dV
 * and E_FG = 3/5 N eF of the uniform gas of the same mean density.
 * Quasi-1D integrals include the transverse area. */
tdslda_status tdslda_energy(tdslda_ctx* ctx, double terms_out[9]);

/* Conservation check of Sec. 4.5.1 against the values at the first call
 * after a load (or after tdslda_set_external): returns EUNSTABLE if
 * |N-N0|/N0 > tol_N, |Omega-Omega0|/E_FG > tol_E with Omega = E_total - mu N
 * (the quantity of Eq. E_tot, conserved at fixed mu), or a state norm is not
 * finite.  The N check is skipped while Delta_ext is non-zero.  out[3] (may
 * be NULL) = {dN/N0, dOmega/E_FG, max |norm - 1|}. */
tdslda_status tdslda_check(tdslda_ctx* ctx, double out[3]);

/* Copy the current normalised states to the host ([n][2][M][2] FP64). */
tdslda_status tdslda_get_states(tdslda_ctx* ctx, double* uv);
/* Current state count, steps taken since load, elapsed time. */
tdslda_status tdslda_info(tdslda_ctx* ctx, int64_t* nstates, int64_t* steps, double* time);

/* Checkpoint / resume (Sec. 4.5.1): states, integrator history, per-state
 * scalars, weights, fields and the step counter, written raw in the context
 * precision.  tdslda_load requires a context created with the same lattice,
 * precision, integrator and capacity >= the saved state count. */
tdslda_status tdslda_save(tdslda_ctx* ctx, const char* path);
tdslda_status tdslda_load(tdslda_ctx* ctx, const char* path);

/* Streaming device-to-device copy of `bytes` bytes on hip_stream (a
 * hipStream_t; NULL = the null stream), asynchronous: 128-bit non-temporal
 * loads and stores, consecutive lanes on consecutive words.  The HBM
 * reference of the measurement (a plain read-once / write-once kernel of
 * known traffic); also used by the stationary start-up to replicate the
 * history.  dst and src are device pointers, 16-byte aligned, not
 * overlapping; bytes >= 0 is a multiple of 16.  Errors: EINVAL (alignment,
 * size, overlap), EDEVICE (launch failure). */
tdslda_status tdslda_device_copy(void* dst, const void* src, int64_t bytes, void* hip_stream);

/* Streaming read of `bytes` bytes of src on hip_stream (NULL = the null
 * stream), asynchronous: 128-bit non-temporal loads, consecutive lanes on
 * consecutive words, nothing written (sink16, a 16-byte device buffer, is
 * written only for one particular data pattern, to keep the loads).  The
 * read-only HBM reference of the measurement, beside tdslda_device_copy.
 * src and sink16 16-byte aligned device pointers; bytes a multiple of 16.
 * Errors: EINVAL (alignment, size), EDEVICE (launch failure). */
tdslda_status tdslda_device_read(const void* src, int64_t bytes, void* sink16, void* hip_stream);

/* Kernel timing.  With profiling on, every kernel launch is bracketed by HIP
 * events on the context stream; tdslda_kernel_stats returns, for kernel class
 * k (see tdslda_kernel_name), the launch count and the summed milliseconds
 * since the last reset.  Returns EINVAL for k out of range. */
tdslda_status tdslda_set_profiling(tdslda_ctx* ctx, int enable);
tdslda_status tdslda_kernel_stats(tdslda_ctx* ctx, int k, int64_t* launches, double* total_ms);
const char* tdslda_kernel_name(int k); /* NULL past the last class */

#ifdef __cplusplus
}
#endif
#endif /* TDSLDA_H */
