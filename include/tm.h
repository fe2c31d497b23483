/*
 * tm.h -- C ABI of the MI355X Liouville-Lanczos magnon library (libtm).
 *
 * Method: Liouville-Lanczos time-dependent density-functional perturbation
 * theory for spin-wave spectra, arXiv:2203.01120 (Gorni, Baseggio, Delugas,
 * Baroni, Timrov).  The library computes, on one AMD Instinct MI355X
 * (gfx950), the Liouvillian-times-vector product of Sec. 2.4
 * (Eqs. Liouvillian_BR_q and liouvillian_blocks), the two Lanczos recursions
 * of Sec. 2.5 built on it, and the susceptibility of Eqs.
 * resolvent_Liouvillian_Lanczos_q and post_processing.
 *
 * Units: Hartree atomic units (bohr, Ha), as in Sec. 2.1.  Spin density
 * m = psi^dag sigma psi (mu_B = 1).
 *
 * Conventions shared by every call:
 *   - complex numbers are two consecutive doubles (re, im);
 *   - a lattice-periodic spinor component is
 *       U(r) = Omega^{-1/2} sum_G c(G) exp(i G.r),  G = m1 b1 + m2 b2 + m3 b3,
 *     with coefficient arrays laid out [band][spin][G] (spin 0 = up) in the
 *     order of the Miller list given for that point;
 *   - grid fields are C-order [n1][n2][n3] on r = (i1/n1) a1 + (i2/n2) a2 + (i3/n3) a3;
 *   - a batch-representation (BR) vector of q-set iq is complex
 *       [2 sides][nk][nbnd][2 spins][npw_pad]
 *     (side 0 = X, side 1 = Y of Eq. batch_rho), each (side, k) block on the
 *     plane-wave sphere of the point k+q of mesh point k, in the Miller order
 *     of that point, zero-padded to npw_pad (see tm_qset_info; one value for
 *     every q set of a system: the longest k+q sphere of all of them, rounded
 *     up to 16);
 *   - inner product (a, b) = (1/nk) sum conj(a) b.
 *
 * Errors: every call returns an int, TM_OK (0) on success and a negative
 * code otherwise; tm_last_error() gives a message for the calling thread.
 * Nothing here falls back to the CPU: a missing or unusable GPU is TM_EDEVICE.
 */
#ifndef TM_H
#define TM_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TM_OK = 0,
    TM_EINVAL = -1,       /* invalid argument or inconsistent input data        */
    TM_ENOMEM = -2,       /* device allocation failed                           */
    TM_EDEVICE = -3,      /* HIP runtime or kernel launch error                 */
    TM_EBREAKDOWN = -4,   /* Lanczos breakdown: result holds the valid prefix   */
    TM_EUNSUPPORTED = -5  /* size outside what the kernels support (e.g. grid
                             length with a prime factor other than 2, 3, 5)     */
};

/*
 * Arithmetic of a Liouvillian application (Eq. liouvillian_blocks).
 * TM_FP64: everything in double precision.
 * TM_FP32 (single-precision bulk): the 3D FFTs, the response densities, the
 *   real-space products and the nonlocal/projector contractions (FP32 MFMA,
 *   FP32 accumulation) run in single precision; the Hartree + xc potential,
 *   the kinetic term, the BR vectors themselves, every Lanczos recurrence and
 *   inner product and chi stay FP64, and the chains re-project their vectors
 *   onto the empty manifold in FP64 every step.  Needs the fixed-size plane
 *   and z kernels and the resident real-space ground state
 *   (tm_system_set_resident_limit), else TM_EUNSUPPORTED at the first apply.
 */
typedef enum { TM_FP64 = 0, TM_FP32 = 1 } tm_precision;

/* Direction of the perturbing field (Sec. 2.5, Eq. off-diag-resolvent):
 * sigma^mu = sigma_x, sigma_y, sigma_z, sigma_x + i sigma_y, sigma_x - i sigma_y,
 * and TM_DIR_N = sigma_0, the charge channel of the generalized 4 x 4
 * (charge + spin) susceptibility (Sec. 2.3).  sigma_0 is even under time
 * reversal where the spin matrices are odd, so its vectors carry the opposite
 * sign on the lower (y) side: u^n = (U~, +T U~), v^n = (P U~, -P+ T U~). */
typedef enum {
    TM_DIR_X = 0, TM_DIR_Y = 1, TM_DIR_Z = 2, TM_DIR_PLUS = 3, TM_DIR_MINUS = 4, TM_DIR_N = 5
} tm_dir;

/* Lanczos flavour (Sec. 2.5): non-Hermitian biorthogonalisation (two
 * applications of L per step) or pseudo-Hermitian (one per step). */
typedef enum { TM_NONHERMITIAN = 0, TM_PSEUDOHERMITIAN = 1 } tm_flavour;

typedef struct tm_system tm_system;

/*
 * Description of one system: the ground state of Secs. 2.2 and 3.1 and the
 * q-points to study.  All pointers are host memory owned by the caller; they
 * are read during tm_system_create only and may be freed afterwards.
 *
 * Ground-state points: every k-related point that any q-set needs (k, -k,
 * k+q, -k-q of Sec. 5.7's "sister points") carries its occupied spinors
 * U_{n,p} (all nbnd of them, the lowest), eigenvalues and projector table.
 */
typedef struct {
    double cell[9];             /* lattice vectors a1, a2, a3 as rows (bohr)              */
    int fft[3];                 /* n1, n2, n3: lengths with prime factors 2, 3, 5 only    */
    int nbnd;                   /* occupied spinor bands per k                            */

    int npts;                   /* number of ground-state points                          */
    const double* xk;           /* [npts][3] Cartesian point vectors (bohr^-1)            */
    const int* npw;             /* [npts] sphere sizes                                    */
    const int* const* mill;     /* [npts] -> [npw][3] Miller indices                      */
    const double* const* evc;   /* [npts] -> complex [nbnd][2][npw] occupied spinors      */
    const double* const* et;    /* [npts] -> [nbnd] eigenvalues (Ha)                      */

    const double* vrs;          /* [4][n1 n2 n3]: v_eff, B_x, B_y, B_z of Eq. H0_k_plus_q,
                                   with the Hamiltonian's magnetic term written +B.sigma  */
    const double* rho;          /* [4][n1 n2 n3]: ground-state n, m_x, m_y, m_z            */

    int nproj;                  /* Kleinman-Bylander projectors in the cell                */
    const double* const* vkb;   /* [npts] -> complex [nproj][npw]: beta_i(p+G)            */
    const double* dvan;         /* complex [nproj][nproj][2][2]: spinor D matrix; must be
                                   Hermitian and time-reversal invariant (Sec. 2.2)       */

    int nq;                     /* number of q-sets                                       */
    const double* xq;           /* [nq][3] Cartesian q (bohr^-1)                           */
    int nk;                     /* mesh points per q-set (weights 1/nk)                   */
    const int* roles;           /* [nq][nk][4]: point index of k, -k, k+q, -k-q            */
    const int* shifts;          /* [nq][nk][4][3] or NULL: integer g with
                                   role vector = xk[point] + g.b; the point's
                                   coefficients then sit on Miller indices m - g          */
} tm_system_desc;

/* Per-q-set shape information for sizing BR vectors. */
typedef struct {
    int nk;                     /* mesh points                                            */
    int nbnd;                   /* bands                                                  */
    int npw_pad;                /* padded sphere length of every (side, k) block (the same
                                   for every q set of the system)                          */
    long long nelem;            /* complex elements of one BR vector = 2 nk nbnd 2 npw_pad */
    double lam;                 /* scale of L used by the breakdown rule: the largest
                                   |k+q+G|^2/2 on the response spheres (Ha)               */
} tm_qset_info;

/*
 * tm_system_create: upload a system to the current HIP device and build the
 * G-vector maps, FFT column tables, time-reversed partners (T = i sigma_y K,
 * Sec. 2.2), the ALSDA kernel fields (Eqs. v_XC_q, b_XC_q) and the Coulomb
 * multipliers 4 pi / |G+q|^2 (Eq. v_H_q).
 * Returns TM_EINVAL for inconsistent input (e.g. the sphere of -k-q is not the
 * negative of the sphere of k+q) and for a NaN or Inf in any floating-point
 * input (checked on the host before the device is touched), TM_EUNSUPPORTED
 * for unsupported grid sizes (a length with a prime factor other than 2, 3, 5,
 * or planes of more than 4096 points; also checked before the device is
 * touched), TM_ENOMEM / TM_EDEVICE for device failures.  *out owns all device
 * memory.
 */
int tm_system_create(const tm_system_desc* desc, tm_system** out);

/* Free everything tm_system_create allocated.  NULL is allowed.  TM_EINVAL
 * (nothing freed) while chains of the system exist (tm_chain_end them first). */
int tm_system_destroy(tm_system* sys);

/* Shape of the BR vectors of q-set iq. */
int tm_qset_info_get(const tm_system* sys, int iq, tm_qset_info* info);

/*
 * Resident ground state (a memory/time trade, not part of the method).  Every
 * apply of L (Eq. liouvillian_blocks) needs each ground-state band U_k, and
 * T U_-k on the Y side, in real space.  When the (n1, n2) plane has a
 * fixed-size kernel and the real-space copy fits in `bytes`, the first apply
 * transforms each band once and keeps it in device memory (complex FP64,
 * [distinct (point, G shift, side)][band][i3][spin][n1 n2]); otherwise every
 * apply repeats the in-plane inverse transforms from the bands' z-transformed
 * columns.  Both paths give the same result up to rounding order.
 * bytes < 0 (the default) allows up to 80% of the device memory free at the
 * first apply; 0 disables the copy.  Setting a limit frees an existing copy and
 * the next apply decides again.  Must not be called while work of this system
 * is in flight; TM_EINVAL while chains of the system exist (their captured
 * steps hold the copy's address).  The first apply of a q set after creation
 * or after this call builds these caches and synchronises its stream.
 */
int tm_system_set_resident_limit(tm_system* sys, long long bytes);

/* Bytes of device memory held by the resident real-space ground state (0 if none). */
int tm_system_resident_bytes(const tm_system* sys, long long* bytes);

/*
 * Device memory of a system (an implementation figure, not part of the
 * method): what a scheduler needs to admit work by device-memory footprint.
 *   tables            ground-state bands, occupied partners, projector and
 *                     sphere tables, fields: allocated by tm_system_create
 *   resident          resident real-space ground state now held
 *   resident_full     bytes the complete resident copy needs (0 when the grid
 *                     has no fixed-size plane kernel)
 *   columns           z-transformed ground-state columns now held (the path
 *                     without the resident copy)
 *   columns_full      bytes those columns need for the largest q set
 *   workspace         apply workspaces of every chain slot now held
 *   workspace_per_rhs one slot's workspace for one right-hand side (a chain
 *                     of L lanes needs about L times this in each slot)
 *   chain_slots       workspace slots the system's chains are spread over
 * out: caller-owned host struct.  TM_EINVAL on a null argument.
 */
typedef struct {
    long long tables, resident, resident_full, columns, columns_full, workspace, workspace_per_rhs;
    int chain_slots;
} tm_memory_info;
int tm_system_memory(const tm_system* sys, tm_memory_info* out);

/*
 * The same figures for a system not yet created, from its descriptor alone
 * (host work only, nothing is allocated): resident_full, columns_full and
 * workspace_per_rhs as tm_system_memory will report them; tables an upper
 * estimate (its items summed, 5 % and 1 MiB added); the "now held"
 * fields and chain_slots are 0.  TM_EINVAL on a null or empty descriptor;
 * TM_EUNSUPPORTED for a grid tm_system_create refuses (a length with a prime
 * factor other than 2, 3, 5, or planes of more than 4096 points).
 */
int tm_system_footprint(const tm_system_desc* desc, tm_memory_info* out);

/*
 * tm_liouvillian_apply: xy_out = L_q xy_in (Eqs. Liouvillian_BR_q and
 * liouvillian_blocks; one projector P, P+ applied to the sum of the D and K
 * parts, lower row multiplied by -1).
 * xy_in, xy_out: device pointers to BR vectors of q-set iq (see tm_qset_info),
 * owned by the caller; they must not overlap (TM_EINVAL).  The padding of
 * xy_in must be zero; xy_out's padding is written as zero.  The input should
 * be orthogonal to the occupied manifold (X side to U_{k+q}, Y side to
 * T U_{-k-q}); the output always is.
 * stream: a hipStream_t (NULL = default stream); the call is asynchronous.
 * prec: TM_FP64 or TM_FP32 (see tm_precision).
 */
int tm_liouvillian_apply(tm_system* sys, int iq, const void* xy_in, void* xy_out,
                         tm_precision prec, void* stream);

/*
 * tm_liouvillian_apply_multi: nrhs (1..4) applications in one pass.  xy_in and
 * xy_out hold nrhs BR vectors back to back (vector r at + r * nelem complex
 * elements); the kernels take the right-hand sides as extra batches, reading
 * the ground state and the projector and occupied-state tables once for all.
 * Each output equals tm_liouvillian_apply of its input bit for bit.  Grows the
 * system's workspace to nrhs right-hand sides (see tm_chain_begin_multi).
 */
int tm_liouvillian_apply_multi(tm_system* sys, int iq, int nrhs, const void* xy_in, void* xy_out,
                               tm_precision prec, void* stream);

/*
 * Autotuning of launch shapes (an implementation device, not part of the
 * method).  Several launches of the apply exist as compiled variants that
 * split the same work differently: the plane density and apply kernels
 * (butterflies per load group, columns per wave, row loads in flight), the z
 * passes (threads, columns and items per block), the projector / P_c
 * contractions (K split) and their updates (loads grouped ahead of the
 * products or not).  Before a system's first tunable launch -- its
 * first FP64 apply, start vector with a projection (tm_start_vectors with
 * v), FP64 chain begin or restore -- outside a stream capture, every variant
 * is timed on that system's data (the first apply's own vectors, else two
 * scratch vectors allocated and freed for the purpose) and the fastest is
 * kept for that shape for the rest of the process; later systems of the same
 * shape reuse it.  So every result of a system comes from the same variants,
 * whichever call came first.  The plane and z-pass launches of several
 * right-hand sides (lanes) are timed again, on the caller's vectors, at the
 * system's first FP64 apply of that many (one size class per power of two):
 * their best shapes change once the grid fills the device.  Their variants
 * give identical results, so this changes no result; the contractions and
 * updates keep the one-right-hand-side choice.  Plane, z-pass and update
 * variants give identical results; the contraction variants sum K in
 * different splits (results equal up to
 * rounding), so two processes may differ in the last bits -- forcing the
 * contraction variant (tm_autotune_force(4, 0)) makes results reproducible
 * bit for bit across processes, e.g. for a chain saved in one and restored in
 * another.  A first call issued under stream capture is not timed (timing
 * needs synchronisation); the system is tuned at its next such call outside
 * a capture, and launches captured before that keep the variants in force
 * when they were captured.
 *   tm_autotune_enable(on): on (the default) or off (variant 0, the
 *     hand-picked default, for shapes not yet tuned).
 *   tm_autotune_force(op, variant): use `variant` of operation op for every
 *     shape (op: 0 plane density, 1 plane apply, 2 z inverse, 3 z forward,
 *     4 contraction, 5 update); -1 returns to the tuned choice.  A variant beyond a
 *     shape's count makes that apply fail with TM_EINVAL.  For tests.
 *   tm_autotune_report(buf, cap, needed): the tuned shapes as text, one line
 *     each: operation, shape, number of variants, chosen variant, measured
 *     microseconds per variant (tab-separated).  Writes at most cap bytes
 *     (NUL-terminated) to the caller's buf (may be NULL) and the full size in
 *     *needed.
 */
int tm_autotune_enable(int on);
int tm_autotune_force(int op, int variant);
int tm_autotune_report(char* buf, size_t cap, size_t* needed);

/*
 * tm_liouvillian_apply_noalloc: tm_liouvillian_apply (one right-hand side,
 * same kernels, same result) for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  It calls no hipMalloc, hipFree or allocating routine: its apply
 * workspace is a static device array of 64 MiB inside the library, one copy
 * per device, held until the process ends.  Systems whose one-right-hand-side
 * workspace (tm_system_memory's workspace_per_rhs, rounded up per buffer) is
 * larger get TM_EUNSUPPORTED (the 20^3 / 8-band system needs about 7 MB).
 * The q set's ground-state caches must already exist -- one ordinary
 * tm_liouvillian_apply of that q set builds them -- else TM_EINVAL; the
 * current device must be the system's (TM_EINVAL).  Every call on a device
 * shares that device's array, which keeps the last call's contents; calls
 * that overlap on one device (other streams, other threads) race and must be
 * serialised by the caller.  Arguments, layout and the other errors as for
 * tm_liouvillian_apply.
 */
int tm_liouvillian_apply_noalloc(tm_system* sys, int iq, const void* xy_in, void* xy_out,
                                 tm_precision prec, void* stream);

/*
 * tm_start_vectors: the BR vectors of Sec. 2.5 (below Eq. off-diag-resolvent):
 *   u^dir = ( sigma U~_{n,k}, -sigma T U~_{n,-k} ),
 *   v^dir = ( P sigma U~_{n,k}, P+ sigma T U~_{n,-k} ),
 * U~ = coefficients restricted to the sphere of k+q.  u, v: device BR vectors
 * (either may be NULL).  Asynchronous on stream, except that with v on a
 * system not yet tuned it first builds the ground-state caches and runs the
 * autotuner (see tm_autotune_enable), which synchronises.
 */
int tm_start_vectors(tm_system* sys, int iq, tm_dir dir, void* u, void* v, void* stream);

/*
 * Lanczos coefficients (Sec. 2.5).  All arrays are host memory owned by the
 * caller with room for `capacity` steps.  For 0-based step j:
 *   alpha[j] = T[j][j], beta[j] = T[j+1][j], gamma[j] = T[j][j+1],
 *   z[l][j] = (u^l, q_j) for l = x, y, z;  zn[j] = (u^n, q_j) (charge);
 * the last beta/gamma is the residual coupling beyond the M x M matrix.
 * For the pseudo-Hermitian flavour beta = gamma (real) and alpha is real.
 * zn may be NULL (then the charge overlaps are not returned).
 */
typedef struct {
    int capacity;               /* in: room for this many steps                          */
    int steps_done;             /* out: steps whose alpha and z are valid                */
    double n1;                  /* out: norm of the start vector used (Sec. 2.5)         */
    double* alpha;              /* complex [capacity]                                    */
    double* beta;               /* real    [capacity]                                    */
    double* gamma;              /* complex [capacity]                                    */
    double* z;                  /* complex [3][capacity]                                 */
    double* zn;                 /* complex [capacity] or NULL                             */
} tm_coeffs;

/*
 * tm_lanczos_run: one chain for field direction dir on q-set iq, nsteps
 * steps (nsteps <= out->capacity), flavour f.  Synchronous.  Breakdown rule
 * (scale Lam from tm_qset_info, eps = 1e-10):
 *   non-Hermitian: |(p^, q^)| <= eps Lam^2 ||p_i|| ||q_i||;
 *   pseudo-Hermitian start: v^dag J L v <= eps Lam (v, v);
 *   pseudo-Hermitian step:  r^dag J L r <= eps Lam (r, r) or (r, r) <= eps^2 Lam^2 (q_i, q_i).
 * On breakdown the call returns TM_EBREAKDOWN with steps_done < nsteps and
 * the coefficients of the completed steps valid.
 */
int tm_lanczos_run(tm_system* sys, int iq, tm_dir dir, tm_flavour f, int nsteps,
                   tm_precision prec, tm_coeffs* out);

/*
 * tm_tensor_run: tm_lanczos_run for ndir directions at once (1..4, e.g. x, y,
 * z for the 3 x 3 spin tensor or n, x, y, z for the 4 x 4 one), stepped
 * together as the lanes of one chain (see tm_chain_begin_multi); out: ndir
 * tm_coeffs, each as tm_lanczos_run fills it.  TM_EBREAKDOWN if any lane
 * broke down (the others ran all nsteps).  Synchronous.
 */
int tm_tensor_run(tm_system* sys, int iq, int ndir, const tm_dir* dirs, tm_flavour f, int nsteps,
                  tm_precision prec, tm_coeffs* out);

/*
 * Chain-level interface (serving).  One chain = one recursion of Sec. 2.5 for
 * (q set, direction, flavour), resident on the device; tm_lanczos_run is
 * begin + steps + coeffs + end.
 * tm_chain_begin: allocates the chain's vectors (pseudo-Hermitian: 5 BR
 *   vectors, non-Hermitian: 9, plus the four u^lambda, lambda = x, y, z, n) and coefficient
 *   storage for `capacity` steps, builds v^mu (as tm_start_vectors) and
 *   starts the recursion (pseudo-Hermitian: one apply), asynchronously on
 *   `stream` (a hipStream_t, NULL = default stream).  TM_ENOMEM when the
 *   vectors do not fit.
 * tm_chains_step: advances each of the n chains by up to k_steps steps (never
 *   past its capacity), one step per chain in turn, ordered on `stream`;
 *   asynchronous.  Chains may belong to different systems, but all work of
 *   one system must be issued on one stream at a time (its chains share the
 *   system's apply workspaces).  The chains of a system whose apply
 *   workspace is small (at most 256 MB) are spread over up to 3 workspace
 *   slots (see tm_system_set_chain_slots): slot 0 runs on `stream`, the other
 *   slots on library streams that wait for the work issued on `stream` before
 *   the call and that `stream` waits for before anything issued after it, so
 *   the chains of different slots overlap on the device.  The step index and
 *   the breakdown flag live on the device: after a breakdown the chain's
 *   coefficients stop changing.
 * tm_chain_coeffs: waits for the chain's last stream, copies the first
 *   min(capacity, out->capacity) coefficients, steps_done and n1 into `out`
 *   (layout of tm_coeffs; one struct per lane, see below); TM_EBREAKDOWN
 *   when a lane has broken down.
 * tm_chain_end: waits for the chain's last stream and frees it (NULL allowed).
 *
 * Several field directions in one pass (the full tensor; ipol = 4 of
 * turbo_magnon, Table 1): tm_chain_begin_multi starts one chain with ndir
 * lanes (1 <= ndir <= 4), one independent recursion per direction dirs[r].
 * The lanes step together: every application of L, every projection and
 * every inner product runs once for all lanes, with the lanes as extra
 * batches of the same kernels (the ground state and the projector and
 * occupied-state tables are read once per step for all of them).  Each lane's
 * coefficients equal those of a single-direction chain bit for bit; a lane
 * that breaks down idles while the others go on.  tm_chain_lanes returns the
 * lane count; tm_chain_coeffs then takes an array of that many tm_coeffs.
 * The system's apply workspace grows to ndir right-hand sides (its
 * reallocation makes other chains of the system re-capture their graphs).
 * tm_chain_begin is tm_chain_begin_multi with one direction.
 *
 * Many chains in one launch (a q path, Sec. 5: the spectra of many q, each
 * a chain of its own): tm_chain_begin_lanes starts one chain with nlanes
 * lanes (1..96), lane r the recursion for q set iqs[r] and direction
 * dirs[r] (the same q set may appear in several lanes).  Every step runs each
 * kernel once for all lanes -- z passes, plane kernels, potential, nonlocal
 * and projector contractions, update and inner products -- with the lanes as
 * extra batches: each batch reads the sphere, column, plane-row and resident
 * ground-state tables of its lane's q set from tables laid out lane after
 * lane (built once per distinct list iqs, kept with the system), and each
 * lane has its own measure vectors u^lambda.  Each lane's coefficients equal
 * those of a single chain of its q set and direction bit for bit.  Lanes of
 * different q sets need the resident real-space ground state (fixed-size
 * plane kernels and room for it; TM_EUNSUPPORTED otherwise).  The BR vectors
 * of every q set of a system have one layout (the spheres are padded to the
 * longest of all q sets; tm_qset_info_get), so lane r's vectors sit at
 * r nelem in each of the chain's buffers.  The system's apply workspace
 * grows to nlanes right-hand sides.  tm_chain_begin_multi is
 * tm_chain_begin_lanes with every lane on q set iq.
 */
typedef struct tm_chain tm_chain;
/* Steps are replayed from a captured HIP graph of one period of steps (6
 * pseudo-Hermitian, 3 non-Hermitian) when possible; tm_chains_use_graphs(0)
 * issues every kernel directly (process-wide switch, default on; the kernel
 * profiler also issues directly).  Both give identical coefficients. */
int tm_chains_use_graphs(int on);
int tm_chain_begin(tm_system* sys, int iq, tm_dir dir, tm_flavour f, tm_precision prec, int capacity,
                   void* stream, tm_chain** out);
int tm_chain_begin_multi(tm_system* sys, int iq, int ndir, const tm_dir* dirs, tm_flavour f, tm_precision prec,
                         int capacity, void* stream, tm_chain** out);
int tm_chain_begin_lanes(tm_system* sys, int nlanes, const int* iqs, const tm_dir* dirs, tm_flavour f,
                         tm_precision prec, int capacity, void* stream, tm_chain** out);
int tm_chain_lanes(const tm_chain* chain, int* lanes);
int tm_chains_step(tm_chain* const* chains, int n, int k_steps, void* stream);
/* tm_system_set_chain_slots: at most nslots (1..16, default 3) workspace
 * slots for the chains of sys begun afterwards; 1 runs all of them on the
 * caller's stream (for a caller that overlaps systems on streams of its
 * own).  Each slot holds its own apply workspace.  TM_EINVAL while chains of
 * sys exist or for nslots outside 1..16. */
int tm_system_set_chain_slots(tm_system* sys, int nslots);
int tm_chain_coeffs(tm_chain* chain, tm_coeffs* out);
int tm_chain_end(tm_chain* chain);

/*
 * Chain checkpoint and restart (the restart / restart_step inputs of
 * turbo_magnon, Sec. 3.2 and Table 1): the chain's complete state -- its BR
 * vectors, the three u^lambda, the coefficients and the device scale/step
 * state -- as one host blob.
 * tm_chain_state_size: bytes of the blob (per lane 5 BR vectors pseudo-Hermitian
 *   or 9 non-Hermitian and 104 bytes per step of capacity, plus the 4 measure
 *   vectors -- shared, or per lane when the lanes carry different q sets --
 *   and a header).
 * tm_chain_save: waits for the chain's last stream and copies its state into
 *   `host` (caller-owned, at least tm_chain_state_size bytes); the chain stays
 *   usable.
 * tm_chain_restore: a new chain of system `sys` from a blob saved from a chain
 *   of the same system (same q set shapes; TM_EINVAL otherwise), with
 *   capacity max(capacity, saved capacity) -- a restart may run more steps
 *   than the original chain was sized for.  Stepping it continues the
 *   recursion exactly where the saved chain stood: the coefficients equal
 *   those of an uninterrupted chain bit for bit.  Synchronises `stream`; the
 *   blob may be released when the call returns.
 */
int tm_chain_state_size(const tm_chain* chain, size_t* bytes);
int tm_chain_save(tm_chain* chain, void* host, size_t bytes);
int tm_chain_restore(tm_system* sys, const void* host, size_t bytes, int capacity, void* stream,
                     tm_chain** out);

/*
 * tm_chi: chi_l(omega_j) = n1 sum_i z[l][i] eta_i with
 *   ((omega_j + i eta) I - T) eta = e_1            (Eq. post_processing)
 * over the first m_use steps (m_use <= c->steps_done), l = x, y, z.
 * omega: host [nomega] (Ha); chi: host complex [3][nomega], caller-owned.
 * Runs on the current device (one tridiagonal solve with partial pivoting per
 * frequency); synchronous.
 */
int tm_chi(const tm_coeffs* c, int m_use, const double* omega, int nomega, double eta,
           double* chi);

/*
 * tm_chi_extrapolated: tm_chi on a tridiagonal matrix extended from m_use
 * computed steps to m_total (Sec. 2.5, last paragraph on the Lanczos
 * algorithm; the turbo_spectrum inputs itermax0 = m_use, itermax = m_total,
 * extrapolation = 'constant' | 'osc' of Sec. 3.3 and Table 2).  The paper names
 * the schemes without formulas; this library's reading: past m_use, alpha,
 * beta and gamma take their mean over the second half of the computed
 * coefficients (indices m_use/2 .. m_use-1) -- one mean (TM_EXTRAP_CONSTANT)
 * or one per parity of the index (TM_EXTRAP_OSC, bi-constant) -- and z is
 * zero (no overlaps were measured there).  TM_EXTRAP_NONE requires
 * m_total == m_use and equals tm_chi.  m_use >= 4 when extrapolating.
 * Work memory on the device: 64 * m_total * nomega bytes.  Synchronous.
 */
typedef enum { TM_EXTRAP_NONE = 0, TM_EXTRAP_CONSTANT = 1, TM_EXTRAP_OSC = 2 } tm_extrap;
int tm_chi_extrapolated(const tm_coeffs* c, int m_use, int m_total, tm_extrap mode, const double* omega,
                        int nomega, double eta, double* chi);

/*
 * tm_chi_tensor: one column (field direction mu of the chain) of the
 * generalized 4 x 4 susceptibility, rows lambda = n, x, y, z:
 *   chi[0] from zn, chi[1..3] from z, otherwise as tm_chi_extrapolated.
 * c->zn must be set.  chi: host complex [4][nomega].  Synchronous.
 */
int tm_chi_tensor(const tm_coeffs* c, int m_use, int m_total, tm_extrap mode, const double* omega,
                  int nomega, double eta, double* chi);

/*
 * tm_structure_factor: S(q, omega) = -Im Tr[P_perp(q) chi(q, q; omega)]
 * (Eq. S_def), P_perp_ab = delta_ab - q_a q_b / q^2.
 * q: host [3] Cartesian (bohr^-1), nonzero (TM_EINVAL for q = 0).
 * chi: host complex chi_{lambda mu}(omega) at index (lambda * 3 + mu) * nomega
 *   + omega (interleaved re, im); column mu is what tm_chi returns for the
 *   chain with field direction mu (x, y, z).
 * s: host [nomega].  Host arithmetic only; synchronous.
 */
int tm_structure_factor(const double* q, const double* chi, int nomega, double* s);

/*
 * Kernel timing.  While enabled, every kernel launch of the library is
 * bracketed by two HIP events on the stream it runs on; tm_profile_count
 * synchronises the device, folds the elapsed times per kernel name and
 * returns the number of distinct kernels; tm_profile_get(i, ...) returns the
 * name (truncated to name_cap-1 chars), total milliseconds and launch count of
 * entry i (TM_EINVAL when i is out of range).  Process-wide; not thread-safe.
 */
int tm_profile_enable(int on);
int tm_profile_reset(void);
int tm_profile_count(void);
int tm_profile_get(int i, char* name, int name_cap, double* total_ms, long long* launches);

/* Message for the last error on the calling thread ("" if none). */
const char* tm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TM_H */
