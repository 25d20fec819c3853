/* mkpw -- many-k plane-wave Hamiltonian on AMD Instinct MI355X (gfx950).
 *
 * C-ABI of the batched Kohn-Sham H|psi> of Gong & Dal Corso (CPC 2024,
 * arXiv 2412.01695) and of the two solvers built on it.  One context holds
 * one crystal (lattice, cutoff, FFT mesh, k-point list, local potential,
 * projectors) on one GPU; every k-point of the list is processed in the
 * same kernel launches (the paper's "many k" method, Sec. 3, Algorithms
 * new_gpu and phonon_new).
 *
 * Conventions
 *   Units: lengths bohr, energies Hartree, wavefunction cutoff in Ry; the
 *   basis at k is every G with |k+G|^2 < ecutwfc_Ry bohr^-2 (Sec. 2.2.1).
 *   Complex numbers are interleaved (re, im) pairs: complex128 = 2 doubles,
 *   complex64 = 2 floats.
 *   Wavefunction arrays are (nk, nvec, npwx) row-major; row (k, v) holds the
 *   npw[k] coefficients in the library's plane-wave order (ascending
 *   |k+G|^2, ties by Miller index (m1, m2, m3) lexicographically; see
 *   pw_get_miller) followed by npwx - npw[k] padding entries that must be
 *   zero on input and are written as zero on output.
 *   The set-up calls (pw_set_lattice, pw_set_cutoff, pw_set_kpoints,
 *   pw_set_vloc, pw_set_projectors, pw_set_qij) take host arrays only and
 *   copy them to the device once: the potential, the projector rows and the
 *   D and q coefficients are inputs of the crystal, not of each call.  The
 *   per-call vectors (wavefunctions, H|psi>, right-hand sides, solutions,
 *   induced densities) are device memory; the small per-k arrays
 *   (eigenvalues, shifts, weights, iteration counts) and the perturbing
 *   potential of pw_dfpt_rhs are host arrays, as each entry point states.
 *   Device pointers are HIP device memory owned by the caller (e.g. torch
 *   tensors); the library never frees or reallocates them.  All device work
 *   is ordered on the context's stream; calls return once the work is
 *   enqueued unless stated otherwise.  Host pointers are read during the
 *   call only.
 *   Every call returns a pw_status; on error pw_last_error() holds a message
 *   and the context is unchanged unless stated otherwise.  No exception
 *   crosses the ABI.
 *   Threads: a context is used by one host thread at a time; different
 *   contexts may be used from different threads at once.  Besides its device
 *   memory a context keeps a small page-locked host buffer (grown to what the
 *   solvers' per-iteration copies need), freed by pw_destroy.
 */
#ifndef MKPW_H
#define MKPW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pw_ctx pw_ctx;

typedef enum {
  PW_OK = 0,
  PW_EINVAL = -1,  /* invalid argument (message says which) */
  PW_ENOMEM = -2,  /* device allocation failed or HBM budget exceeded */
  PW_EDEVICE = -3, /* HIP runtime error */
  PW_ENOCONV = -4, /* solver stopped at max_iter; results and flags written */
  PW_ESTATE = -5   /* call out of order (e.g. h_psi before set_vloc) */
} pw_status;

typedef enum {
  PW_FP64 = 0, /* complex128 H|psi>, FP64 everywhere */
  PW_MIXED = 1 /* complex64 H|psi> with FP32 accumulation; solvers keep FP64
                  Gram / Rayleigh-Ritz / CG scalars and refine in FP64 */
} pw_prec;

/* Create a context on HIP device `hip_device`, ordering its work on
 * `hip_stream` (a hipStream_t; NULL = a stream owned by the context, created
 * with default priority).  hip_device = -1 makes a host-only context that
 * can build and report the plane-wave basis but runs no device work (every
 * device call then returns PW_ESTATE).  On success *out owns the context. */
pw_status pw_create(pw_ctx** out, int hip_device, void* hip_stream);

/* Free the context and every device buffer it owns.  NULL is a no-op. */
void pw_destroy(pw_ctx* ctx);

/* Message of the last failed call on this context; never NULL. */
const char* pw_last_error(const pw_ctx* ctx);

/* Options: "hbm_budget_bytes" (0 = none; larger device workspaces fail with
 * PW_ENOMEM, the paper's memgpu input of Sec. 5.1), "davidson_basis_factor"
 * (maximum Davidson basis in units of nbnd, default 4, Sec. 5.3), "trace"
 * (nonzero: synchronise and check after every launch), "hpsi_variant"
 * (0 = autotuned on first use, 1 = one work-item per FFT line, 2 = two lanes
 * per line, 3 = two lanes per x line and one per y and z line, 4 = one
 * work-item per line with each x line evaluated as one convolution over the
 * window, 5 = as 4 with two lanes per y and z line; 2, 3 and 5 on even meshes
 * only; 4 and 5 where the window is narrower than the mesh), "hpsi_slab" (0 = autotuned, else the number of z planes
 * transformed together) and "hpsi_threads" (0 = autotuned, else 256, 512 or
 * 1024 work-items per workgroup where the kernel fits in the registers
 * that leaves; PW_EINVAL otherwise).  Any nonzero shape option fixes the
 * shape: the others default to variant 1, 256 work-items and the widest slab
 * that fits.
 * "tune_log" (nonzero: print each autotuning candidate's time to stderr),
 * "solver_graph" (default 1: pw_davidson and pw_dfpt_cg capture one iteration
 * as a HIP graph and replay it; 0: launch every kernel of every iteration
 * one by one; the results are the same), "mixed_refine" (default 1: the
 * PW_MIXED Davidson refines in FP64 after its complex64 phase; 0: it returns
 * the complex64-phase result, for measuring what the refinement adds),
 * "mixed_switch_rtol_e7" (default 2000, in [100, 100000]: the residual norm,
 * in units of 1e-7, below which a band counts as converged in the PW_MIXED
 * Davidson's complex64 phase; the FP64 phase uses 1e-5),
 * "cg_switch_digits" (default 10, in [2, 20]: the PW_MIXED CG leaves complex64
 * once every system's |rho| has fallen by 10^-digits from its start),
 * "dav_nconv" (default 0 = all: pw_davidson declares a k converged once its
 * lowest dav_nconv bands are; the bands above are buffer bands, corrected
 * while the k runs but not waited for, and their results may be less
 * accurate.  A block whose top band is nearly degenerate with the next
 * eigenvalue converges that band slowly; a few buffer bands remove that). */
pw_status pw_set_option(pw_ctx* ctx, const char* key, int64_t value);

/* Read an option (the keys above), or "hpsi_variant_tuned" / "hpsi_slab_tuned" /
 * "hpsi_threads_tuned" (the shape of this context's last H|psi> launch, 0 if
 * none), "device_bytes" (device memory the context holds now), "overlap"
 * (1 while overlap coefficients q are set, else 0), or the context's sizes:
 * "nk" and "npwx" (0 before pw_set_kpoints), "nproj" (0 without projectors),
 * "fft1", "fft2", "fft3" (the mesh; 0 before pw_set_cutoff), and what the
 * last pw_davidson or pw_dfpt_cg did: "last_iterations" (iterations run),
 * "last_hpsi_kbands" (H applications, one per (k, vector) row each time H is
 * applied to it), "last_graph_replays" (iterations run as graph replays). */
pw_status pw_get_option(const pw_ctx* ctx, const char* key, int64_t* value);

/* Direct lattice, rows a1, a2, a3 in bohr (host, 9 doubles).  Resets the
 * basis, potential and projectors. */
pw_status pw_set_lattice(pw_ctx* ctx, const double a[9]);

/* Wavefunction cutoff (Ry) and FFT mesh N1, N2, N3 (host, 3 ints; all zero
 * = smallest 2,3,5-smooth N_i >= 2 floor(2 sqrt(ecut) |a_i| / 2pi) + 1).
 * Sec. 4 requires the mesh to hold every G - G'; this library checks the
 * weaker condition it needs, that each k's sphere fits the mesh without
 * two plane waves sharing a mesh point (else PW_EINVAL). */
pw_status pw_set_cutoff(pw_ctx* ctx, double ecutwfc_ry, const int fft[3]);

/* k-point list: nk Cartesian vectors (host, nk*3 doubles, bohr^-1).  Builds
 * the plane-wave sphere of every k (Sec. 2.2.1) and the FFT-mesh maps of
 * Sec. 4.  Writes npw[k] to npw_out (host, nk ints, may be NULL) and the
 * row length npwx (max npw rounded up to 64) to npwx_out (may be NULL).
 * Resets the projectors. */
pw_status pw_set_kpoints(pw_ctx* ctx, int nk, const double* k_cart, int32_t* npw_out, int32_t* npwx_out);

/* Miller indices of the plane waves of k-point ik in the library's order
 * (host, npw[ik]*3 ints); ik = -1 writes every k-point's list, concatenated
 * in k order (host, sum_k npw[k]*3 ints). */
pw_status pw_get_miller(const pw_ctx* ctx, int ik, int32_t* miller);

/* Local potential V_eff(r) on the FFT mesh (Sec. 2.2.2, Sec. 4): host
 * array of N1*N2*N3 real doubles in Ha, C order (l3 fastest), point
 * l = (l1, l2, l3) at r = sum_i l_i / N_i a_i. */
pw_status pw_set_vloc(pw_ctx* ctx, const double* v_r);

/* Nonlocal pseudopotential (Sec. 2.2.3): projector values beta_p(k+G)
 * (host, complex128 (nk, nproj, npwx), library plane-wave order, padding
 * ignored) and the coefficients D_pq (host, complex128 nproj x nproj,
 * Hermitian to 1e-12 relative, else PW_EINVAL).  nproj = 0 removes the
 * nonlocal term.  nproj <= 32. */
pw_status pw_set_projectors(pw_ctx* ctx, int nproj, const void* beta, const void* dij);

/* Overlap coefficients q_pq (Sec. 2.2, overlap operator of ultrasoft and PAW
 * pseudopotentials): S = 1 + sum_pq |beta_p> q_pq <beta_q| with the
 * projectors of pw_set_projectors.  qij: host complex128 nproj x nproj,
 * Hermitian to 1e-12 relative (else PW_EINVAL); NULL removes the overlap
 * (S = 1).  Needs projectors (nproj > 0) set first (else PW_ESTATE);
 * pw_set_projectors and pw_set_kpoints remove it.  With an overlap set,
 * pw_davidson solves H psi = eps S psi and pw_dfpt_cg uses
 * A = H - eps S + alpha S P_v S.  S must be positive definite (it is when q
 * is positive semidefinite); the solvers report PW_EINVAL when the basis
 * Gram matrix in the S inner product is not. */
pw_status pw_set_qij(pw_ctx* ctx, const void* qij);

/* Random starting vectors for pw_davidson, drawn on the device:
 * psi(k, b, G) = (x + i y) / (1 + |k+G|^2/2), normalised per band, x and y
 * two N(0, 1) values (Box-Muller) from the SplitMix64 finaliser chained over
 * (seed, k, b, packed Miller index (m1+512)<<20 | (m2+512)<<10 | (m3+512));
 * the value at a plane wave does not depend on the batch or the order.
 * psi: device complex128 (nk, nbnd, npwx), padding written as zero. */
pw_status pw_init_guess(pw_ctx* ctx, int nbnd, uint64_t seed, void* psi);

/* Hpsi = H psi for every k-point and band at once (Sec. 3, H application):
 * kinetic (1/2)|k+G|^2 psi, local potential (scatter -> inverse 3D FFT ->
 * V(r) -> forward 3D FFT with 1/N_r -> gather) and nonlocal
 * sum_pq beta_p D_pq <beta_q|psi> (Eqs. lambdah, gamma, finalnl).
 * psi and hpsi: device, (nk, nbnd, npwx); complex128 for PW_FP64,
 * complex64 for PW_MIXED; they must not overlap.
 * The transforms are compiled for cubic meshes N^3 with N in {15, 18, 20, 24,
 * 30, 32, 36} (the 2,3,5-smooth sizes of cutoffs up to about 60 Ry for cells
 * like the workloads here); any other mesh is refused with PW_EINVAL, as every
 * entry point that applies H does. */
pw_status pw_h_psi(pw_ctx* ctx, pw_prec prec, int nbnd, const void* psi, void* hpsi);

/* pw_h_psi for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation):
 * the same H|psi>, arguments and result as pw_h_psi, but the call allocates
 * nothing, times nothing and synchronises nothing.  What the kernel reads of
 * the potential (V permuted for its slab width, or the taps of its x-line
 * convolutions) is staged in a fixed array of the library (808 704 bytes, one
 * per GPU, held until the process ends; PW_EINVAL for a mesh that needs
 * more), rebuilt on every call.  The launch shape is the one
 * pw_h_psi has tuned for this mesh and batch size if it has, else a fixed
 * default (no tuning).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams or threads) race. */
pw_status pw_h_psi_noalloc(pw_ctx* ctx, pw_prec prec, int nbnd, const void* psi, void* hpsi);

/* Spsi = S psi for every k-point and band at once (Sec. 2.2 overlap
 * operator, Eqs. lambdah, delta_eq, finals): psi + sum_p delta_p beta_p with
 * delta_p = sum_q q_pq <beta_q|psi>; a copy of psi when no overlap is set.
 * psi and spsi: device, (nk, nbnd, npwx); complex128 for PW_FP64,
 * complex64 for PW_MIXED (FP32 arithmetic); spsi may be psi itself (in
 * place), otherwise they must not overlap.  Padding written as zero. */
pw_status pw_s_psi(pw_ctx* ctx, pw_prec prec, int nbnd, const void* psi, void* spsi);

/* Lowest nbnd eigenpairs of H psi = eps S psi at every k by block Davidson
 * (Sec. 2.1; S = 1 without an overlap), all k-points advancing together,
 * each stopping on its own.  1 <= nbnd <= 32 (else PW_EINVAL); the basis
 * holds at most min(4 nbnd, 64) vectors per k (the reduced problems are
 * solved in LDS; option "davidson_basis_factor" sets the 4), and a k whose
 * next block would exceed it restarts from its Ritz vectors.
 * psi: device complex128 (nk, nbnd, npwx): starting vectors in, eigenvectors
 * out (S-orthonormal).  eig_ha: host (nk, nbnd) doubles, eigenvalues in Ha.
 * A k-point is converged when every band's (with option "dav_nconv", every
 * one of the lowest dav_nconv bands') eigenvalue changed by less than
 * tol_ry/2 Ha in the last iteration and its residual norm |H psi - e S psi| is
 * below 1e-5 (so the eigenvalue error is of order residual^2 / gap).
 * iters, converged: host (nk) ints, may be NULL.
 * PW_MIXED applies H in complex64 until every band's eigenvalue changes by
 * less than max(tol_ry/2, 2e-6) Ha with residual norm below 2e-4 (what an
 * FP32 H application resolves; option "mixed_switch_rtol_e7"), then refines with H in FP64 to the FP64
 * criterion above (option "mixed_refine" = 0 stops after the complex64 phase).
 * Every per-iteration decision (which bands get a correction, restarts,
 * dropped blocks) is taken on the device; the host only learns, one iteration
 * late, whether any k is still active.
 * Returns PW_ENOCONV if some k did not converge within max_iter. */
pw_status pw_davidson(pw_ctx* ctx, pw_prec prec, int nbnd, void* psi, double* eig_ha, double tol_ry,
                int max_iter, int32_t* iters, int32_t* converged);

/* Batched preconditioned CG (Sec. 2.4) for the DFPT linear systems
 * (Eq. linear_system at q = 0 with the valence projector of Eq. projector):
 * (H - eps_{k,nu} S + alpha_k S P_v S) x_{k,nu} = rhs_{k,nu},
 * P_v = sum_{mu<nocc} |u_mu><u_mu|, one system per (k, nu), nu < nrhs
 * (S = 1 without an overlap).
 * psi_occ: device complex128 (nk, nocc, npwx) S-orthonormal u.
 * eps_ha: host (nk, nrhs) doubles.  alpha_ha: host (nk) doubles, > 0.
 * rhs: device complex128 (nk, nrhs, npwx).  dpsi: device complex128
 * (nk, nrhs, npwx): initial guess in, solution out.
 * Preconditioner M_GG = max(1, (|k+G|^2/2) / <psi_nu|T|psi_nu>) with psi_nu
 * = psi_occ row nu (nrhs <= nocc) (Sec. 2.4).  Each system stops when
 * |rho| = |Re <M^-1 r|r>| < thr; converged systems are frozen.
 * iters: host (nk*nrhs) ints (updates applied to each system), may be NULL.
 * PW_MIXED applies H in complex64 while the residual update and all scalars
 * stay FP64, until every system's |rho| has dropped by 1e-10 from its start
 * (option "cg_switch_digits"), then recomputes the residual with H in FP64 and
 * continues to thr.
 * Returns PW_ENOCONV if some system did not converge within max_iter updates
 * (both phases of PW_MIXED together). */
pw_status pw_dfpt_cg(pw_ctx* ctx, pw_prec prec, int nocc, const void* psi_occ, const double* eps_ha,
               const double* alpha_ha, int nrhs, const void* rhs, void* dpsi, double thr, int max_iter,
               int32_t* iters);

/* Right-hand sides of the DFPT linear systems at a wavevector q (Sec. 2.3,
 * Eq. linear_system with dS = 0; Algorithm phonon_new, "build P_c dV u"):
 *   rhs_{k,nu} = -(1 - S P_v^{k+q}) dV u_{k,nu},
 *   (dV u)(G') = sum_G dV~[(m_G' - m_G) mod N] u(G),  G on the k sphere,
 *   G' on the k+q sphere, dV~ the forward transform of dV(r) with 1/N_r.
 * ctx_kq holds the k+q list (k-point i = k_i + q), ctx_k the k list, on the
 * same device, lattice and mesh with the same number of k-points (else
 * PW_EINVAL); work runs on ctx_kq's stream (ctx_k must have no pending work).
 * dv_r: host complex128 N1*N2*N3 (C order), the lattice-periodic part of the
 * perturbing potential in Ha.  psi_k: device complex128 (nk, nocc, npwx_k),
 * the occupied states at k.  psi_occ_kq: device complex128 (nk, nocc,
 * npwx_kq), the S-orthonormal occupied states at k+q (S of ctx_kq).
 * rhs: device complex128 (nk, nocc, npwx_kq), written (padding zero); feed it
 * to pw_dfpt_cg on ctx_kq with psi_occ_kq and the eigenvalues at k.
 * 1 <= nocc <= 64.  FP64. */
pw_status pw_dfpt_rhs(pw_ctx* ctx_kq, const pw_ctx* ctx_k, int nocc, const void* dv_r, const void* psi_k,
                const void* psi_occ_kq, void* rhs);

/* Density induced by a perturbation at q (Sec. 2.3, Eq. drho without the
 * augmentation term):  drho(r_l) = 4 sum_k w_k sum_nu conj(u_{k,nu}(r_l))
 * du_{k,nu}(r_l), with u(r_l) = sum_G u(G) exp(2 pi i m_G . l / N) (the
 * inverse transform of Sec. 4, no normalisation).  Contexts as for
 * pw_dfpt_rhs.  wk: host (nk) k-point weights.  psi_k: device complex128
 * (nk, nbnd, npwx_k).  dpsi_kq: device complex128 (nk, nbnd, npwx_kq), the
 * solutions of pw_dfpt_cg (in the conduction manifold).  drho_r: device
 * complex128 N1*N2*N3 (C order), written.  1 <= nbnd <= 1024.  FP64.
 * The pair sums of a k are added into their Miller-difference bins with
 * atomics, so the order of additions varies: repeated calls agree to rounding,
 * not bit for bit.
 * PW_EINVAL if the spheres are too large for the difference bins held in LDS
 * (more than about 9000 distinct Miller differences per x-plane). */
pw_status pw_drho(pw_ctx* ctx_kq, const pw_ctx* ctx_k, int nbnd, const double* wk, const void* psi_k,
            const void* dpsi_kq, void* drho_r);

#ifdef __cplusplus
}
#endif

#endif /* MKPW_H */
