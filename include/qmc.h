/*
 * qmc.h -- C ABI of the batched JAGP (Jastrow x antisymmetrized geminal power)
 * wave-function library for AMD Instinct MI355X (gfx950).
 *
 * What is computed (arXiv:2002.07401, TurboRVB review):
 *   Psi(x)   = det(W) exp(J)                    (Wave functions section; eq:wfAGPs)
 *   W[i][j]  = sum_{mu,nu} Lambda[mu][nu] psi_mu(r_i) psi_nu(r_j),
 *              i an up electron, j a down electron          (agp_expansion)
 *   psi_mu   = P_{l,m}(r - R_a) exp(-zeta_mu |r - R_a|^2)   (eq. gaussian)
 *   J        = J1 + J2                    (onebody_J_hom, onebody_u, twobody_jastrow,
 *                                          twobody_v)
 *   e_L      = (H Psi)/Psi, H the all-electron Coulomb Hamiltonian in Hartree
 *              units                       (local energy, Variational Monte Carlo section)
 *   ratio    = Psi(x')/Psi(x) for x' differing from x by one electron; QMC cost is
 *              set by e_L and by such ratios (Wave functions section, intro).
 *
 * Conventions shared by every call:
 *   - Electrons 0..n_up-1 are spin up, n_up..N-1 spin down (AGP section ordering).
 *   - Real solid harmonics P_{l,m}, unnormalised, component index m:
 *       l=0: 1;  l=1: x, y, z;  l=2: xy, yz, zx, x^2-y^2, 2z^2-x^2-y^2.
 *   - Arrays are row-major, FP64 unless stated.  "Device" pointers point to memory
 *     of the GPU that is current when the call is made; the caller owns them.
 *     Every call that takes a stream enqueues its work on that stream and
 *     returns without waiting (create/destroy and qmc_walkers_read's host copy
 *     excepted).
 *   - A handle may be used by one host thread at a time; distinct handles are
 *     independent.
 *   - Errors: a negative qmc_status.  Argument and shape errors are detected
 *     on the host before anything is enqueued, and qmc_last_error() returns a
 *     thread-local message.  HIP launch errors surface as QMC_ERR_HIP.  Per-walker
 *     numerical problems never fail a call; they are reported in status[w]:
 *        0 ok, 1 singular geminal matrix (det = 0), 2 non-finite result,
 *        3 refreshed on drift: a periodic refresh replaced an inverse whose
 *          residual max|W X - I| exceeded the walker set's drift tolerance
 *          (qmc_walkers_set_drift_tol).  The inverse diverges where det W
 *          vanishes (the Atomic forces section relates G^{-1} to 1/Pf near
 *          nodes), so this flags walkers near a node.
 */
#ifndef QMC_JAGP_H
#define QMC_JAGP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QMC_ABI_VERSION 19

typedef enum {
  QMC_OK = 0,
  QMC_ERR_ARG = -1,         /* null pointer, out-of-range index or enum        */
  QMC_ERR_SHAPE = -2,       /* sizes the library cannot handle                 */
  QMC_ERR_HIP = -3,         /* a HIP runtime call failed                       */
  QMC_ERR_OOM = -4,         /* device allocation failed                        */
  QMC_ERR_UNSUPPORTED = -5, /* a feature of the description is not built       */
  QMC_ERR_STATE = -6        /* call order violated (e.g. accept before propose) */
} qmc_status;

/* Arithmetic of the geminal products (W build, move rows) and of the stored
 * basis matrices.  LU, inverse, inverse updates and ratio accumulation are
 * FP64 in every mode. */
typedef enum {
  QMC_FP64 = 0,    /* everything FP64                                           */
  QMC_W_FP32 = 1,  /* Phi, P = Phi Lambda and the W products in FP32 on MFMA
                      with FP32 accumulation; FP64 LU/inverse/SM/ratios          */
  QMC_MIXED = 2,   /* moves as QMC_W_FP32 (FP32 Phi and P rows streamed by the
                      proposals); every qmc_eval_batch builds Phi, P, W and the
                      cofactor products in FP64 (log|Psi|, E_loc and drift at
                      FP64 accuracy) and stores the FP32 copies the moves read.
                      Two extra [Wk][N][round_up(L,32)] FP64 work arrays.        */
  QMC_MIXED_BF16 = 3, /* as QMC_MIXED with the moves' Phi and P rows stored in
                      BF16 (half the streamed bytes of FP32; the P half rebuilds
                      between evaluations run on MFMA from the BF16 rows with
                      FP32 accumulation); ratios and updates FP64              */
  QMC_W_BF16 = 4,  /* unrefined geminal build on BF16 matrix instructions with
                      FP32 accumulation (not built: QMC_ERR_UNSUPPORTED)        */
  QMC_W_FP8 = 5,   /* unrefined geminal build on FP8 matrix instructions (not
                      built: QMC_ERR_UNSUPPORTED)                              */
  QMC_REFINED = 6  /* the mixed path held to the FP64 oracle: every P = Phi Lambda
                      product (evaluation and the P rebuilds between moves) on
                      the int8 matrix cores as an error-free digit expansion
                      (7 int8 digits per FP64 row, exact int32 accumulation:
                      error below 7e-14 of max|Phi| max|Lambda| L); Phi, P, W,
                      LU, inverse, cofactors, ratios and updates FP64;
                      proposals stream only the P columns of basis functions
                      whose value at r' can change the determinant ratio:
                      those skipped contribute at most 1e-13 in total (bound
                      from the largest |P| of each column and the inverse
                      column's 1-norm; an up move of a polarized system also
                      streams the unpaired orbitals' values).  One more
                      [Wk][L][N + n_up - n_dn] FP64
                      array (P transposed).  For a Pfaffian (pairing = 1) the
                      evaluation's B rows phi(r_j)^T K^{s s_j} are the same
                      error-free int8 digit products; G~, Pf, its inverse and
                      the moves are those of the FP64 path.                    */
} qmc_precision;

typedef struct qmc_system qmc_system;   /* opaque: nuclei, basis, Lambda, Jastrow */
typedef struct qmc_walkers qmc_walkers; /* opaque: per-walker state for moves     */

/* System description.  All pointers are HOST pointers; the arrays are copied
 * to the device by qmc_system_create and may be freed afterwards. */
typedef struct {
  int32_t n_nuc;              /* number of nuclei A                              */
  const double *R;            /* [A][3] nuclear positions (bohr)                 */
  const double *Z;            /* [A] nuclear charges                             */
  int32_t n_basis;            /* L                                               */
  const int32_t *center;      /* [L] nucleus index of each basis function        */
  const int32_t *l;           /* [L] angular momentum, 0..2                      */
  const int32_t *m;           /* [L] component index (see above)                 */
  const int32_t *radial;      /* [L] 0 Gaussian e^{-zeta r^2} (eq. gaussian),
                                 1 Slater e^{-zeta r} (eq. slater)                */
  const double *zeta;         /* [L] exponents                                   */
  const double *lambda;       /* [L][L] pairing coefficients (general matrix;
                                 symmetric for a spin singlet)                   */
  int32_t n_up, n_dn;         /* electrons per spin, n_up >= n_dn (label the
                                 majority spin "up")                             */
  int32_t j1_form;            /* 0 none, 1 u=(1-e^{-bs})/(2b), 2 u=s/(2(1+bs))   */
  const double *j1_b;         /* [A] one-body b per nucleus                      */
  int32_t j2_form;            /* 0 none, 1 Pade (b_para, b_anti),
                                 2 Pade series (b,a1,a2,a3 parallel, then anti)  */
  int32_t n_j2;               /* 2 for form 1, 8 for form 2                      */
  const double *j2;           /* [n_j2]                                          */
  int32_t precision;          /* qmc_precision                                   */
  int32_t refresh_every;      /* recompute W^{-1} from W after this many
                                 attempted moves of one spin (>= 1; at most 64
                                 are buffered, see qmc_accept_move)              */
  /* Jastrow basis chi_k (same function kinds as the geminal basis) for the
   * one-body inhomogeneous and three/four-body terms (onebody_J_inh,
   * threebody_jastrow):
   *   J1inh = sum_i sum_k j1_inh[s_i][k] chi_k(r_i)
   *   J3/4  = sum_{i<j} sum_{k,l} chi_k(r_i) M^{s_i s_j}[k][l] chi_l(r_j)
   * Up electrons come first, so unlike-spin pairs i < j use M^{ud}; the
   * same-spin matrices must be symmetric.  n_jbasis = 0: no such terms.
   * Not supported with them: qmc_multi_*.  qmc_system_set_jastrow_basis
   * replaces the coefficients and exponents. */
  int32_t n_jbasis;           /* LJ <= 1024                                      */
  const int32_t *jb_center;   /* [LJ] nucleus index                              */
  const int32_t *jb_l;        /* [LJ] 0..2                                       */
  const int32_t *jb_m;        /* [LJ] component index                            */
  const int32_t *jb_radial;   /* [LJ] 0 Gaussian, 1 Slater (may be NULL: all 0)  */
  const double *jb_zeta;      /* [LJ]                                            */
  const double *j1_inh;       /* [2][LJ] coefficients for up, then down electrons */
  const double *j3;           /* [3][LJ][LJ] M^{uu}, M^{dd} (symmetric), M^{ud}   */
  /* Contracted orbitals (Contraction of the primitive atomic basis section):
   * with n_contracted = Lc > 0 the L basis functions above are primitives and
   * the geminal is built from phi_c = sum_t con_coef[t] psi_{con_idx[t]} over
   * t in [con_ptr[c], con_ptr[c+1]), c < Lc; lambda is then [Lc][Lc] and every
   * [L] of the calls below that refers to orbitals (Phi rows) reads Lc.
   * L <= 2048 primitives.  qmc_forces returns the gradients with respect to the
   * primitives' exponents, Lambda over the contracted orbitals and con_coef
   * (qmc_grads.dcon_coef).  Not supported with it: qmc_multi_*. */
  int32_t n_contracted;       /* Lc (0: the basis functions are the orbitals)    */
  const int32_t *con_ptr;     /* [Lc + 1], con_ptr[0] = 0, non-decreasing        */
  const int32_t *con_idx;     /* [con_ptr[Lc]] primitive index, 0 .. L-1         */
  const double *con_coef;     /* [con_ptr[Lc]] coefficients                      */
  /* Unpaired orbitals (eq:wfAGPunpaired): with k = n_up - n_dn > 0 the geminal
   * matrix is n_up x n_up, columns n_dn + l holding sum_mu unpaired[mu][l]
   * phi_mu(r_i) (phi the orbitals: the basis functions, or the contracted
   * orbitals).  Not supported with it: qmc_multi_*; qmc_forces returns the
   * gradient with respect to them in qmc_grads.dunpaired. */
  const double *unpaired;     /* [L or Lc][k]; may be NULL when k = 0            */
  /* Pfaffian pairing (Pfaffian wave function section), pairing = 1: Psi =
   * Pf(G~) exp J with G~_ij = phi(r_i)^T A^{s_i s_j} phi(r_j) (eq:g,
   * agp_expansion), A^{ud} = lambda (singlet plus triplet-zero part, any
   * matrix), A^{du} = -lambda^T, A^{uu} = pf_uu and A^{dd} = pf_dd
   * skew-symmetric; pf_k unpaired orbitals as fictitious electrons
   * (eq:pfodd): G~_{i, N+l} = phi(r_i) . U^{s_i}[:, l] with U^u = unpaired
   * and U^d = pf_unpaired_dn.  N + pf_k must be even and at most 96;
   * precision QMC_FP64 or QMC_REFINED; n_up < n_dn is allowed.  Not supported with it:
   * qmc_multi_*.  qmc_reweight uses G~ and its inverse;
   * qmc_system_set_params (lambda = A^{ud}) and qmc_system_set_pfaffian change
   * the coefficients. */
  int32_t pairing;            /* 0 AGP determinant, 1 Pfaffian                   */
  const double *pf_uu;        /* [L][L] skew-symmetric                           */
  const double *pf_dd;        /* [L][L] skew-symmetric                           */
  int32_t pf_k;               /* unpaired orbitals of the Pfaffian               */
  const double *pf_unpaired_dn; /* [L][pf_k]                                     */
} qmc_system_desc;

/* Version of this header the library was built from (QMC_ABI_VERSION). */
int32_t qmc_abi_version(void);

/* Message of the last failed call on this host thread ("" if none). */
const char *qmc_last_error(void);

/* Copy a description to the current device.  Fails with QMC_ERR_UNSUPPORTED
 * for l > 2, n_up < n_dn or a precision not built. */
qmc_status qmc_system_create(const qmc_system_desc *desc, qmc_system **out);
qmc_status qmc_system_destroy(qmc_system *sys);

/* Replace parameters of a system from DEVICE arrays (any may be NULL to keep
 * the current values): R [A][3], zeta [n_basis], lambda [L][L], jas [A + n_j2]
 * (one-body b per nucleus, then the two-body parameters).  Work is enqueued on
 * `stream` and the call returns without waiting (every parameter, the two-body
 * ones included, is read by the kernels from device memory).  Walker sets of
 * this system must be re-evaluated (qmc_eval_batch) before further moves:
 * proposals return QMC_ERR_STATE until then. */
qmc_status qmc_system_set_params(qmc_system *sys, const double *R, const double *zeta,
                                 const double *lambda, const double *jas, hipStream_t stream);

/* Replace the Jastrow-basis coefficients and exponents from DEVICE arrays (any
 * may be NULL to keep the current values): j1_inh [2][LJ], j3 [3][LJ][LJ]
 * (M^{uu}, M^{dd}, M^{ud}; the same-spin blocks must be symmetric, which is not
 * checked here), jb_zeta [LJ].  Enqueued on `stream`; walker sets must be
 * re-evaluated before further moves.  QMC_ERR_ARG without a Jastrow basis. */
qmc_status qmc_system_set_jastrow_basis(qmc_system *sys, const double *j1_inh, const double *j3,
                                        const double *jb_zeta, hipStream_t stream);

/* Replace the Pfaffian's same-spin blocks and unpaired orbitals from DEVICE
 * arrays (any may be NULL): pf_uu, pf_dd [L][L] (skew-symmetric, not checked
 * here), unpaired, unpaired_dn [L][pf_k].  A^{ud} changes through
 * qmc_system_set_params' lambda.  Walker sets must be re-evaluated.
 * QMC_ERR_ARG for a determinant system. */
qmc_status qmc_system_set_pfaffian(qmc_system *sys, const double *pf_uu, const double *pf_dd,
                                   const double *unpaired, const double *unpaired_dn, hipStream_t stream);

/* Flags of a walker set. */
#define QMC_WALKERS_ADJOINT 1   /* reserve the reverse-pass workspace of qmc_forces */

/* Bytes of device memory a walker set of n_walkers walkers of sys occupies
 * with these flags: positions, basis matrix Phi, P = Phi Lambda, W, W^{-1},
 * move buffers and, with QMC_WALKERS_ADJOINT, the reverse-pass workspace.
 * Every later call on the walker set works inside this memory (no call
 * other than create allocates). */
qmc_status qmc_workspace_size(const qmc_system *sys, int32_t n_walkers, int32_t flags, size_t *bytes);

/* Create the device state of n_walkers walkers of sys.  ws: caller-owned
 * DEVICE memory of at least qmc_workspace_size bytes, 256-byte aligned, that
 * the walker set uses until it is destroyed (the library never frees it); or
 * NULL, and the library allocates that much once.  The memory is cleared here
 * (this call synchronises the device).  The state is undefined until
 * qmc_eval_batch has run.  QMC_ERR_ARG for a smaller or misaligned ws. */
qmc_status qmc_walkers_create(qmc_system *sys, int32_t n_walkers, int32_t flags, void *ws, size_t ws_bytes,
                              qmc_walkers **out);
qmc_status qmc_walkers_destroy(qmc_walkers *wk);

/* Tolerance of the drift check made by every refresh that qmc_accept_move
 * triggers with a status array: the inverse about to be replaced, X, is
 * multiplied by W and status[w] = 3 where max|W X - I| > tol (for walkers the
 * refresh found non-singular).  tol < 0 turns the check off; the default is
 * 1e-6.  The last residuals are readable as QMC_STATE_RESIDUAL. */
qmc_status qmc_walkers_set_drift_tol(qmc_walkers *wk, double tol);

/* Evaluate every walker from scratch at positions r and make that the walkers'
 * state.  (Local energy definition, VMC section; eq:wfAGPs; agp_expansion.)
 *   r      [Wk][N][3]  device, read; or NULL: the walkers' current positions
 *                      (those of the last evaluation with the moves accepted
 *                      since).  Then, in QMC_FP64, QMC_W_FP32 and QMC_REFINED,
 *                      the P rows of a spin none of whose electrons has been
 *                      proposed since the rows were last built are reused (the
 *                      rebuild between the halves of a sweep leaves the up rows
 *                      current for the next evaluation); QMC_ERR_STATE before
 *                      the first evaluation.
 *   logabs [Wk]        device, write: log|Psi|
 *   sign   [Wk]        device, write: sign(Psi) = sign(det W); 0 when singular
 *   drift  [Wk][N][3]  device, write, may be NULL: grad_i log|Psi|
 *   e_kin  [Wk]        device, write, may be NULL: -1/2 sum_i lap_i Psi / Psi
 *   e_loc  [Wk]        device, write, may be NULL: e_kin + Coulomb potential
 *   status [Wk]        device, write, may be NULL
 * Resets the move counter used by refresh_every. */
qmc_status qmc_eval_batch(qmc_system *sys, qmc_walkers *wk, const double *r,
                          double *logabs, double *sign, double *drift,
                          double *e_kin, double *e_loc, int32_t *status,
                          hipStream_t stream);

/* Propose moving electron `electron` of every walker to r_new[w] and return
 * ratio[w] = Psi(x')/Psi(x) (signed).  The determinant factor comes from the
 * new row (up electron) or column (down electron) of W contracted with the
 * matching column/row of W^{-1} (one row or column of the geminal matrix
 * changes when one electron moves, Wave functions section).
 *   r_new     [Wk][3] device, read
 *   ratio     [Wk]    device, write
 *   drift_new [Wk][3] device, write, may be NULL: grad log|Psi| of the moved
 *             electron at its new position
 * A second propose replaces the first. */
qmc_status qmc_propose_move(qmc_system *sys, qmc_walkers *wk, int32_t electron,
                            const double *r_new, double *ratio, double *drift_new,
                            hipStream_t stream);

/* Accept (accept[w] != 0) or reject the pending proposal of `electron` for
 * every walker: on accept, new row/column of W, new basis row and position,
 * and a rank-1 update of W^{-1} (FP64) held in delayed form: the inverse of the
 * last refresh A0 plus buffers V, D and S^{-1} of the moves since, with
 * W^{-1} = A0 - V S^{-1} D^T A0 (up moves; transposed for down moves), equal
 * to successive Sherman-Morrison updates (McDaniel et al., J. Chem. Phys. 147,
 * 174107, 2017).  After min(refresh_every, 64) attempted moves of one spin,
 * and before proposing an electron of the other spin while moves are
 * buffered, W^{-1} and log|det W| are recomputed from W by FP64 elimination.
 * QMC_ERR_STATE if no proposal of this electron is pending.
 *   accept [Wk] device, read (uint8)
 *   status [Wk] device, write, may be NULL: written when this accept triggers
 *          a refresh (1 when it finds det = 0, 3 when the replaced inverse had
 *          drifted, see qmc_walkers_set_drift_tol, else 0), untouched otherwise */
qmc_status qmc_accept_move(qmc_system *sys, qmc_walkers *wk, int32_t electron,
                           const uint8_t *accept, int32_t *status, hipStream_t stream);

/* Run n_steps Metropolis single-electron steps (VMC section): step t moves
 * electron (e_start + t) mod N of every walker by disp[t][w] and accepts iff
 * unif[t][w] < ratio^2 (strict), all on the device.
 *   disp         [n_steps][Wk][3] device, read
 *   unif         [n_steps][Wk]    device, read
 *   accept_count [Wk]             device, read-write, may be NULL: += accepted */
qmc_status qmc_vmc_steps(qmc_system *sys, qmc_walkers *wk, int32_t e_start, int32_t n_steps,
                         const double *disp, const double *unif, int32_t *accept_count,
                         hipStream_t stream);

/* Outputs of qmc_forces (device pointers; any may be NULL to skip it).
 * n_jas = n_nuc (one-body b per nucleus) + n_j2 (two-body parameters). */
typedef struct {
  double *dR;       /* [A][3] summed over walkers, or [Wk][A][3] per walker      */
  double *dzeta;    /* [n_basis] or [Wk][n_basis] (the primitives' exponents)    */
  double *dlambda;  /* [L][L] or [Wk][L][L]: d/dLambda[mu][nu], every entry
                       independent (the caller applies any symmetry constraint) */
  double *djas;     /* [n_jas] or [Wk][n_jas]                                    */
  double *dr;       /* [Wk][N][3] (always per walker)                            */
  /* Jastrow basis (n_jbasis = LJ > 0; ignored otherwise): */
  double *dj1_inh;  /* [2][LJ] or [Wk][2][LJ]                                    */
  double *dj3;      /* [3][LJ][LJ] or [Wk][3][LJ][LJ]: M^{uu}, M^{dd} as gradients
                       with respect to symmetric matrices (written symmetric:
                       dF = sum_kl D_kl dM_kl for every symmetric dM); M^{ud}
                       every entry independent                                  */
  double *djb_zeta; /* [LJ] or [Wk][LJ]                                          */
  /* Unpaired orbitals (k = n_up - n_dn > 0; ignored otherwise): */
  double *dunpaired; /* [L][k] or [Wk][L][k]: d/dU[mu][l], U as in the descriptor */
  /* Contracted orbitals (n_contracted > 0; ignored otherwise): */
  double *dcon_coef; /* [nnz] or [Wk][nnz], nnz = con_ptr[n_contracted]: d/dcon_coef[t] */
  /* Pfaffian systems (pairing = 1; must be NULL otherwise): dlambda is A^{ud},
   * dunpaired the up spin's unpaired orbitals [L][pf_k]; the skew same-spin
   * blocks as gradients with respect to skew matrices (written skew), and the
   * down spin's unpaired orbitals: */
  double *dpf_uu;    /* [L][L] or [Wk][L][L]                                       */
  double *dpf_dd;    /* [L][L] or [Wk][L][L]                                       */
  double *dunpaired_dn; /* [L][pf_k] or [Wk][L][pf_k]                              */
} qmc_grads;

/* Adjoint of the evaluation (Derivatives of energy section: logarithmic
 * derivatives O_k of the wave function and derivatives of the local energy,
 * all obtained by one reverse pass).  For every walker w it differentiates
 *     F_w = gbar_logpsi[w] * log|Psi_w| + gbar_eloc[w] * e_L,w
 * with respect to the nuclear positions, basis exponents, pairing matrix,
 * Jastrow parameters and electron positions.  per_walker = 0 sums the
 * parameter gradients over walkers (a vector-Jacobian product); 1 returns
 * them per walker.  r [Wk][N][3] device; gbar_* [Wk] device, NULL means 0.
 * Re-evaluates the walkers at r (their state becomes that of qmc_eval_batch).
 * FP64 systems with <= 256 nuclei (any electron count the evaluation takes,
 * up to 2048).  Needs a walker set
 * created with QMC_WALKERS_ADJOINT (QMC_ERR_STATE otherwise); allocates
 * nothing.
 * Pfaffian systems: every output above (log|Psi| through the cofactor
 * vectors Y_i, e_L through Y, G~^{-1} and the pairing rows), the pairing
 * coefficients in dlambda (A^{ud}), dpf_uu, dpf_dd, dunpaired and dunpaired_dn;
 * with gbar_eloc NULL these equal qmc_pfaffian_logderiv's weighted by
 * gbar_logpsi.  dpf_uu, dpf_dd or dunpaired_dn on a determinant system:
 * QMC_ERR_ARG. */
qmc_status qmc_forces(qmc_system *sys, qmc_walkers *wk, const double *r, int32_t per_walker,
                      const double *gbar_logpsi, const double *gbar_eloc, const qmc_grads *out,
                      hipStream_t stream);

/* Space-warp total derivatives (Atomic forces section: correlated sampling
 * with the space-warp coordinate transformation).  With
 * omega_a(r) = kappa_a(r) / sum_b kappa_b(r), kappa_a(r) = |r - R_a|^-4, for
 * every walker w and nucleus a
 *     out[w][a] = dR[w][a] + sum_i omega_a(r_i) dr[w][i]
 *                 (+ 1/2 sum_i grad omega_a(r_i)   when jacobian != 0)
 * i.e. the derivative of a per-walker quantity when the electrons move with
 * the nuclei; jacobian != 0 gives that of log(J^1/2 |Psi|) from the partials
 * of log|Psi|.  dR and dr are qmc_forces' per-walker partials (of e_L or of
 * log|Psi|).  All pointers device, FP64, row-major:
 *   r   [n_walkers][N][3], dR [n_walkers][A][3], dr [n_walkers][N][3],
 *   out [n_walkers][A][3] (written; may not alias the inputs).
 * N <= 1024.  An electron on a nucleus gives a non-finite result. */
qmc_status qmc_swct(qmc_system *sys, int32_t n_walkers, const double *r, const double *dR, const double *dr,
                    int32_t jacobian, double *out, hipStream_t stream);

/* Finite-variance reweighting factor (Atomic forces section): for every
 * walker, from the geminal matrix W and its inverse of the last evaluation,
 *     R = (S sum_ij (W^-1)_ij^2)^-theta,   S = min_i sum_j W_ij^2
 * (W the geminal matrix, or G~ for the Pfaffian),
 *     weight = (R / max(R, eps))^2,
 * the weight that turns averages over the modified sampling back into
 * averages over |Psi|^2 (R is a distance-to-node measure: small near the
 * node).  Needs qmc_eval_batch (or qmc_forces) since the last accepted move
 * (QMC_ERR_STATE otherwise).  theta > 0, eps >= 0.
 *   R      [Wk] device, written
 *   weight [Wk] device, written, may be NULL */
qmc_status qmc_reweight(qmc_system *sys, qmc_walkers *wk, double theta, double eps, double *R, double *weight,
                        hipStream_t stream);

/* Logarithmic derivatives O_k of the Jastrow-basis coefficients
 * (onebody_J_inh, threebody_jastrow) for every walker at its current positions
 * (after qmc_eval_batch and any accepted moves), the SR step's O_k for these
 * parameters:
 *   d_j1_inh [Wk][2][LJ]:      d log Psi / d j1_inh[s][k] = sum_{i of spin s} chi_k(r_i)
 *   d_j3     [Wk][3][LJ][LJ]:  M^{uu}, M^{dd}: 1/2 (X_s X_s^T - sum_{i of s} chi(r_i) chi(r_i)^T)
 *                              (the gradient with respect to a symmetric matrix,
 *                              written symmetric: dlog Psi = sum_kl D_kl dM_kl for
 *                              every symmetric dM); M^{ud}: X_u X_d^T,
 * X_s = sum_{i of spin s} chi(r_i).  Device pointers, either may be NULL.
 * QMC_ERR_ARG without a Jastrow basis. */
qmc_status qmc_jastrow_basis_logderiv(qmc_system *sys, qmc_walkers *wk, double *d_j1_inh, double *d_j3,
                                      hipStream_t stream);

/* Logarithmic derivatives O_k of the Pfaffian's pairing coefficients for every
 * walker at its current state (after qmc_eval_batch and any accepted moves),
 * from d log Pf = 1/2 tr(G~^{-1} dG~):
 *   d_uu, d_dd [Wk][L][L]: d / dpf_uu, d / dpf_dd (the gradient with respect to a
 *                          skew-symmetric matrix, written skew: dlog Psi =
 *                          sum_kl D_kl dA_kl for every skew dA)
 *   d_ud       [Wk][L][L]: d / dlambda (every entry independent)
 *   d_unpaired_up, d_unpaired_dn [Wk][L][pf_k]: d / dunpaired, d / dpf_unpaired_dn
 * Device pointers, any may be NULL.  QMC_ERR_ARG for a determinant system. */
qmc_status qmc_pfaffian_logderiv(qmc_system *sys, qmc_walkers *wk, double *d_uu, double *d_dd, double *d_ud,
                                 double *d_unpaired_up, double *d_unpaired_dn, hipStream_t stream);

/* Bytes of device workspace qmc_sr_step needs (0 for non-positive sizes). */
size_t qmc_sr_workspace_size(int32_t n_samples, int64_t n_params);

/* Stochastic-reconfiguration step (Stochastic reconfiguration section).  From
 * the logarithmic derivatives O [n_samples][n_params] (row-major, device) and
 * local energies e_loc [n_samples] of the samples, with optional weights
 * [n_samples] (NULL: all 1; averages are sum w x / sum w):
 *     Obar = <O>,  S_kl = <(O_k - Obar_k)(O_l - Obar_l)>,
 *     f_k  = -2 <e_L (O_k - Obar_k)>,
 * solves (S + eps diag(S)) delta = f by conjugate gradients preconditioned by
 * the diagonal of S + eps diag(S), without forming S
 * (each iteration streams O twice), stopping when |r| <= tol |f| or after
 * max_iter iterations; the parameter change is dt * delta for a time step dt
 * the caller chooses.  Every sum is taken in a fixed order, so the result is
 * the same on every run.
 *   delta    [n_params] device, written
 *   force    [n_params] device, written, may be NULL
 *   residual [1] device, written, may be NULL: |r| / |f| at exit
 *   work     device, work_bytes >= qmc_sr_workspace_size(n_samples, n_params)
 * The weights must be positive with a positive sum; with max_iter = 0 delta is 0. */
qmc_status qmc_sr_step(int32_t n_samples, int64_t n_params, const double *O, const double *e_loc,
                       const double *weights, double eps, int32_t max_iter, double tol, double *delta,
                       double *force, double *residual, void *work, size_t work_bytes, hipStream_t stream);

/* qmc_sr_step for callers that cannot allocate device memory and cannot hand
 * in a workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same computation and result, with the
 * workspace taken from a fixed 16 MiB array the library keeps on each GPU
 * until the process ends.  Sizes whose qmc_sr_workspace_size exceeds
 * 16777216 bytes are refused with QMC_ERR_SHAPE (e.g. n_params <= 29900 at
 * 4096 samples, <= 262000 at 128).  Allocates nothing.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (on concurrent streams or
 * host threads) race and must be serialised by the caller. */
qmc_status qmc_sr_step_static(int32_t n_samples, int64_t n_params, const double *O, const double *e_loc,
                              const double *weights, double eps, int32_t max_iter, double tol, double *delta,
                              double *force, double *residual, hipStream_t stream);

/* Several systems moved together (uneven electron counts).  Every phase of a
 * Metropolis step (proposal set-up, streaming rows, accept/update, periodic LU
 * refresh) is one persistent launch over (system, walker[, row chunk]) work
 * items ordered by decreasing cost; each member evolves exactly as it would
 * with qmc_vmc_steps alone given the same random numbers.  Members must have
 * the same precision and n_up <= 128 (unpaired orbitals, a Jastrow basis and
 * contracted orbitals are allowed, and QMC_REFINED members); Pfaffian members
 * are refused (QMC_ERR_UNSUPPORTED); at most 32 members.  The handles stay owned
 * by the caller and must outlive the group. */
typedef struct qmc_multi qmc_multi;
qmc_status qmc_multi_create(int32_t n_members, qmc_system *const *systems, qmc_walkers *const *walkers,
                            qmc_multi **out);
qmc_status qmc_multi_destroy(qmc_multi *m);

/* Time the streaming-rows launch for rows-per-work-item in {8, 16, 32} and
 * persistent grid sizes {512 .. 4096} on the current walker state (read-only
 * apart from proposal scratch) and keep the fastest; returns the choice in
 * *rows and *grid (host, may be NULL).  Synchronises. */
qmc_status qmc_multi_autotune(qmc_multi *m, int32_t *rows, int32_t *grid, hipStream_t stream);

/* n_steps Metropolis steps of every walker of every member; member k moves
 * electron (its move count) mod N_k at each step.  disp/unif: host arrays of
 * n_members DEVICE pointers to [n_steps][Wk_k][3] and [n_steps][Wk_k]; when
 * both are NULL the draws come from Philox4x32-10 (key = seed, counter = the
 * member's move count, walker and member index; see qmc_philox_draws).
 * use_graph != 0 (Philox draws only): the whole n_steps sequence is captured
 * once into a HIP graph and replayed by later calls in the same phase (move
 * counts modulo N_k and refresh_every, cached basis products).  Members must
 * have been evaluated. */
qmc_status qmc_multi_vmc_steps(qmc_multi *m, int32_t n_steps, const double *const *disp,
                               const double *const *unif, uint64_t seed, double sigma, int32_t use_graph,
                               hipStream_t stream);

/* The draws the Philox mode of qmc_multi_vmc_steps uses for member `member`
 * at move count `step`: disp [Wk][3] (Box-Muller normals times sigma) and
 * unif [Wk] in [0, 1), device pointers. */
qmc_status qmc_philox_draws(uint64_t seed, int32_t member, int32_t n_walkers, uint64_t step, double sigma,
                            double *disp, double *unif, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Lattice-regularised diffusion Monte Carlo (Lattice regularized Monte Carlo
 * section), with Psi as the guiding function.
 *
 * The lattice kinetic term connects a configuration x with the 6N
 * configurations x' in which one electron i hops by +-a_i along x, y or z, with
 * matrix element -1/(2 a_i^2).  The potential becomes V^a = V +
 * 1/2 sum_i (Delta^a_i - Delta_i) Psi / Psi (lrdmc_potential).  The fixed-node
 * Hamiltonian H^{FN,gamma} adds (1 + gamma) V_sf to the diagonal, V_sf being
 * the sum over hops with Psi(x')/Psi(x) < 0 of |ratio| / (2 a_i^2), and
 * multiplies those hops' elements by -gamma.  The importance-sampled
 * fixed-node Green's function has off-diagonal elements
 * G_{x',x} = ratio / (2 a_i^2) (ratio > 0) or gamma |ratio| / (2 a_i^2)
 * (ratio < 0) (is-green-function); their sum is the rate of leaving x.
 * Hop order (ratios, hop indices): electron-major, then +x, -x, +y, -y, +z, -z.
 * ------------------------------------------------------------------------ */
typedef struct {
  double a;          /* hop length in bohr (> 0); with a double grid, the
                        length near nuclei                                    */
  double a_valence;  /* > 0: double grid (a reading of the section's double-
                        grid scheme): electrons farther than tf_scale Thomas-
                        Fermi lengths 0.8853 Z^{-1/3} bohr from every nucleus
                        hop by a_valence; <= 0: a everywhere                  */
  double tf_scale;   /* see a_valence (> 0 when a double grid is used)       */
  double gamma;      /* fixed-node spin-flip parameter (>= 0)                 */
} qmc_lrdmc_params;

/* Per-walker terms written by qmc_lrdmc_hops ([Wk][QMC_LR_NTERMS]). */
typedef enum {
  QMC_LR_ELOC = 0,      /* e_L(x) of the last evaluation; equal to the fixed-
                           node lattice local energy sum_x' H^FN_{x',x} Psi(x')/
                           Psi(x) for every gamma (lrdmc_mod_local_energy)   */
  QMC_LR_EKIN = 1,      /* E_kin of the last evaluation                       */
  QMC_LR_LAP_A = 2,     /* sum_i Delta^{a_i}_i Psi / Psi                      */
  QMC_LR_VA_SHIFT = 3,  /* V^a - V                                            */
  QMC_LR_VSF = 4,       /* spin-flip term V_sf                                */
  QMC_LR_ESCAPE = 5,    /* sum of the off-diagonal Green's function elements  */
  QMC_LR_HFN_DIAG = 6,  /* H^{FN,gamma}_{x,x}; the discrete-time diagonal
                           element is lambda minus this, and the column sum
                           b_x = lambda - e_L (lrdmc_mod_weight)              */
  QMC_LR_NTERMS = 7
} qmc_lrdmc_term;

/* Ratios of the 6N lattice hops of every walker and the terms above.  The
 * determinant ratio of a hop of electron i is psi(r')^T y_i with the cofactor
 * row y_i of the last qmc_eval_batch (one row or column of W changes), times
 * exp of the Jastrow change; no inverse is updated.  Needs qmc_eval_batch since
 * the last move of these walkers (QMC_ERR_STATE otherwise); the values of
 * walkers whose status was not 0 are undefined.
 *   params  host pointer
 *   ratios  [Wk][N][6] device, write, may be NULL: Psi(x')/Psi(x)
 *   terms   [Wk][QMC_LR_NTERMS] device, write, may be NULL
 * The walker set keeps both for qmc_lrdmc_advance. */
qmc_status qmc_lrdmc_hops(qmc_system *sys, qmc_walkers *wk, const qmc_lrdmc_params *params,
                          double *ratios, double *terms, hipStream_t stream);

/* One continuous-time step of every walker from the last qmc_lrdmc_hops
 * (treatment of diagonal moves in the Lattice regularized Monte Carlo
 * section).  A walker with tau_left <= 0 or a singular last evaluation is left
 * as it is.  Otherwise it stays in x for tau_xi = -log(1 - xi[w][0]) / escape;
 * if tau_xi >= tau_left its weight is multiplied by exp(-tau_left e_L) and
 * tau_left becomes 0 (no hop); else the weight is multiplied by
 * exp(-tau_xi e_L), tau_left decreases by tau_xi and the walker makes the first
 * hop in hop order whose running sum of Green's function elements exceeds
 * xi[w][1] * escape.  The walkers' own state is not changed: evaluate r_next
 * (qmc_eval_batch) before the next step.
 *   xi       [Wk][2]    device, read: uniforms in [0, 1)
 *   weight   [Wk]       device, read-write
 *   tau_left [Wk]       device, read-write: projection time left
 *   r_next   [Wk][N][3] device, write: positions after the step
 *   hop      [Wk]       device, write, may be NULL: 6 i + direction, or -1 */
qmc_status qmc_lrdmc_advance(qmc_system *sys, qmc_walkers *wk, const double *xi, double *weight,
                             double *tau_left, double *r_next, int32_t *hop, hipStream_t stream);

/* Items of the walker state that qmc_walkers_read can copy out. */
typedef enum {
  QMC_STATE_R = 0,       /* [Wk][N][3]   FP64 positions                          */
  QMC_STATE_LOGABS = 1,  /* [Wk]         FP64 log|Psi| tracked through moves     */
  QMC_STATE_SIGN = 2,    /* [Wk]         FP64 sign(Psi)                          */
  QMC_STATE_W = 3,       /* [Wk][n_up][n_dn] FP64 geminal matrix                 */
  QMC_STATE_AINV = 4,    /* [Wk][n_dn][n_up] FP64 W^{-1} (assembled from the
                            delayed form; uses the walkers' own work arrays)  */
  QMC_STATE_PHI = 5,     /* [Wk][N][L]   FP64 basis values psi_mu(r_i)           */
  QMC_STATE_RESIDUAL = 6, /* [Wk]        max|W X - I| of the last checked refresh
                            (see qmc_walkers_set_drift_tol)                    */
  QMC_STATE_KEPT = 7     /* [Wk]         basis functions the last proposal streamed
                            (QMC_REFINED only; as FP64 values)                */
} qmc_state_item;

/* Copy one item of the walker state into dst (device memory, the layout given
 * above, FP64) on `stream`.  For inspection and checkpoints. */
qmc_status qmc_walkers_read(qmc_walkers *wk, int32_t item, double *dst, hipStream_t stream);

/* Kernel timers.  When timing is enabled on a walker set, every launch the
 * library makes for it is bracketed by a pair of HIP events recorded on the
 * call's stream, and the elapsed times are summed per timer. */
typedef enum {
  QMC_T_BASIS = 0,     /* basis values                                   */
  QMC_T_P_BUILD = 1,   /* P = Phi Lambda of an evaluation (both spins)    */
  QMC_T_W_BUILD = 2,   /* W = P_up Phi_dn^T                              */
  QMC_T_LU = 3,        /* FP64 LU inverse / log-det (eval and refresh)   */
  QMC_T_Y_BUILD = 4,   /* cofactor products for the local energy         */
  QMC_T_ROWDOT = 5,    /* basis-derivative row dots                      */
  QMC_T_ASSEMBLE = 6,  /* Jastrow, Coulomb, local-energy assembly         */
  QMC_T_PROPOSE = 7,   /* proposal, streaming part: new W row/column and
                          the partial determinant ratios                  */
  QMC_T_ACCEPT = 8,    /* Metropolis decision + delayed inverse update   */
  QMC_T_OTHER = 9,     /* small bookkeeping kernels                      */
  QMC_T_PROPOSE_PREP = 10, /* proposal, per-walker part: psi(r'), Jastrow
                              change                                      */
  QMC_T_LRDMC_HOPS = 11,   /* lattice hop ratios and Green's function terms */
  QMC_T_LRDMC_STEP = 12,   /* continuous-time lattice step                  */
  QMC_T_P_REBUILD = 13,    /* one spin's P rows rebuilt before its moves    */
  QMC_T_SWEEP = 14,        /* a run of moves in one persistent launch: the
                              proposals and the accepts fused with the next
                              set-up, between two refreshes               */
  QMC_TIMER_COUNT = 15
} qmc_timer;

/* enable != 0 turns every timer on and clears the sums; 0 turns timing off. */
qmc_status qmc_walkers_set_timing(qmc_walkers *wk, int32_t enable);

/* Turn on only the timers whose bit is set (bit k: timer k of qmc_timer) and
 * clear the sums; 0 turns timing off.  Each timed launch adds two event
 * records to its stream, so a measurement of throughput can time only the
 * kernels it needs. */
qmc_status qmc_walkers_set_timing_mask(qmc_walkers *wk, uint32_t mask);

/* Wait for the recorded events and return, per timer, the summed kernel time in
 * milliseconds (ms[QMC_TIMER_COUNT], host) and the number of launches
 * (launches[QMC_TIMER_COUNT], host).  Synchronises with the recorded events. */
qmc_status qmc_walkers_timing(qmc_walkers *wk, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* QMC_JAGP_H */
