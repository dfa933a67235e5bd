/*
 * lfft — lattice FFT and fast lattice wavelet decomposition for AMD MI355X
 * (gfx950).  C ABI of liblfft.so.
 *
 * Method: R. Bergmann, "The fast Fourier Transform and fast Wavelet Transform
 * for Patterns on the Torus" (arXiv:1107.5415).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - M is a regular integer d x d matrix (1 <= d <= 4), row-major int64,
 *    m = |det M| < 2^31.  Samples are the points y of the pattern P(M),
 *    addressed by their integer key g = M y in G(M) = Z^d / M Z^d
 *    (Section 2.2); frequencies are the classes h of G(M^T).
 *  - NATURAL order of G(M): the box prod_i [0, H_ii) of the column Hermite
 *    normal form H = M U (upper triangular, H_ii > 0, 0 <= H_ij < H_ii for
 *    j > i), enumerated in C order (last coordinate fastest).  NATURAL order
 *    of G(M^T) uses the Hermite form of M^T.  The paper leaves the order of a
 *    pattern open (Section 2.2: any complete set of representatives); this
 *    box is unique for every M.
 *  - GRID order: the lexicographic order of the coefficient vectors lambda
 *    (samples) and mu (frequencies) over Z_eps1 x ... x Z_epsd with respect
 *    to the bases y_j = R^{-1} e_j / eps_j and h_j = R^T e_j of the Smith
 *    form M = Q diag(eps) R (Section 3, eqs. basisPM, basisGM; eq. orderings
 *    of Section 4.1).  In this order the Fourier matrix is the Kronecker
 *    product of 1-D DFTs (Theorem 1) and needs no rearrangement.  Only the
 *    non-trivial eps_j (> 1) are axes; eps is ascending so the largest cycle
 *    is the contiguous axis.
 *  - Data are complex64 (interleaved float re, float im), batch outermost
 *    with stride m.  Masks are float32.
 *  - All buffers passed to execute calls are DEVICE pointers owned by the
 *    caller; the workspace must hold lfft_workspace_size() bytes (may be NULL
 *    when that size is 0).  Execution is out of place (in != out) and ordered
 *    on `stream` (NULL = default stream).  Plans are immutable after
 *    creation and may be used concurrently on different streams only with
 *    distinct workspaces.
 *  - Every function returns LFFT_OK (0) or a negative status; no exception
 *    crosses the ABI.  lfft_strerror() names a status.
 */
#ifndef LFFT_H
#define LFFT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LFFT_OK 0
#define LFFT_E_ARG (-1)          /* null/aliased pointer, bad size or flag    */
#define LFFT_E_SINGULAR (-2)     /* det M = 0                                 */
#define LFFT_E_NOT_INTEGRAL (-3) /* J^{-1} M not integral at some level       */
#define LFFT_E_OVERFLOW (-4)     /* exact integer work would exceed int64     */
#define LFFT_E_UNSUPPORTED (-5)  /* d > 4, m >= 2^31, |det J| > 16, or an
                                    elementary divisor above 2^23 that is no
                                    product of two or three factors of at
                                    most 8192 (shorter ones run as a chirp-z
                                    pass)                                    */
#define LFFT_E_HIP (-6)          /* a HIP call or kernel launch failed        */
#define LFFT_E_NOMEM (-7)        /* device table allocation failed            */
#define LFFT_E_STATE (-8)        /* internal consistency check failed, or an
                                    execute call on a host-only plan          */
#define LFFT_E_IO (-9)           /* a file could not be read or written, or is
                                    not a tuning cache                        */

/* ---- plan log -------------------------------------------------------------
 * With the environment variable LFFT_LOG set to anything but "0" (read once,
 * at the first plan), lfft_plan_create, lwt_plan_create and the lfft_batch_*
 * create/configure/tune calls print the schedule of the plan to stderr: the
 * elementary divisors, the pass count and, per pass of the natural-order
 * forward and inverse transforms, the kernel and its pencil shape; for a
 * pyramid every level's channel grid and which levels are batched. */

/* ---- plan flags --------------------------------------------------------- */
#define LFFT_HOST_ONLY 0x1u      /* integer planning only: no device tables,
                                    execute calls return LFFT_E_STATE         */
#define LFFT_SPLIT_BF16 0x2u     /* lfft_plan_create only: run the radix-16
                                    stages as dense 16-point DFT-matrix
                                    products on BF16 MFMA with split hi+lo
                                    operands and FP32 accumulation
                                    (accuracy bound: 1e-3 relative L2).
                                    Needs power-of-two elementary divisors
                                    and 32 <= m <= 2^24, else UNSUPPORTED    */

#define LWT_SINGLE_STREAM 0x4u   /* lwt_plan_create only: run every kernel of
                                    the pyramid on the caller's stream in issue
                                    order (by default the channel FFTs of the
                                    large levels run on a second, plan-owned
                                    stream that overlaps the splits)         */

#define LWT_SAMPLES 0x8u         /* lwt_plan_create only: the signal side of
                                    the pyramid is point values on P(M), not
                                    coefficients: lwt_decompose changes them
                                    to the orthonormal translates of the
                                    Dirichlet kernel first, lwt_reconstruct
                                    returns point values (lfft_basis_change),
                                    and the adjoints follow               */

/* ---- layouts (bitwise OR of one input and one output choice) ------------ */
#define LFFT_IN_NATURAL 0x0u
#define LFFT_IN_GRID 0x1u
#define LFFT_OUT_NATURAL 0x0u
#define LFFT_OUT_GRID 0x2u

/* ---- index-map selectors ------------------------------------------------ */
#define LFFT_MAP_SAMPLES 0       /* lambda = Q^{-1} g mod eps (forward basis) */
#define LFFT_MAP_FREQS 1         /* mu = R^{-T} h mod eps (forward basis)     */
#define LFFT_MAP_SAMPLES_T 2     /* same for M^T in the inverse basis         */
#define LFFT_MAP_FREQS_T 3

typedef struct lfft_plan_s* lfft_plan_t;
typedef struct lwt_plan_s* lwt_plan_t;

/* Create a lattice-FFT plan for M (row-major d x d) and `batch` signals.
 * Does all integer work on the host, exactly (Section 2.2 Smith form
 * eq. SNF and Hermite boxes; Section 3 bases; Section 4.1 Theorem 1 and
 * Remark 1 for the basis choice) and, unless LFFT_HOST_ONLY, uploads the
 * index and twiddle tables to the current HIP device.  *plan receives the
 * handle (NULL on error).  Errors: ARG, SINGULAR, OVERFLOW, UNSUPPORTED,
 * NOMEM, HIP. */
int lfft_plan_create(lfft_plan_t* plan, int d, const int64_t* M, int64_t batch, uint32_t flags);

/* Release a plan and its device tables (NULL is accepted). */
int lfft_plan_destroy(lfft_plan_t plan);

/* Integer data of the plan (host outputs, any may be NULL):
 * m; d_M = number of eps_j > 1 (Section 2.2); eps[d] ascending with
 * eps_j | eps_{j+1}; Q, R (d x d row-major, unimodular, M = Q diag(eps) R,
 * the forward basis); H_M, H_MT (column Hermite forms of M and M^T). */
int lfft_plan_query(lfft_plan_t plan, int64_t* m, int* d_M, int64_t* eps, int64_t* Q, int64_t* R,
                    int64_t* H_M, int64_t* H_MT);

/* Smith factors M^T = Qt diag(eps) Rt of the basis used by the
 * natural-to-natural inverse (host outputs, d x d row-major each). */
int lfft_plan_query_inverse_basis(lfft_plan_t plan, int64_t* Qt, int64_t* Rt);

/* Number of device passes per transform and whether each basis has its
 * largest cycle aligned with the last sample coordinate (host outputs). */
int lfft_plan_info(lfft_plan_t plan, int* passes, int* aligned_forward, int* aligned_inverse);

/* Host array natural_to_grid[m]: the GRID linear index of every NATURAL
 * index for the selected LFFT_MAP_* (Section 3, eqs. basisPM/basisGM:
 * lambda = Q^{-1} g mod eps, mu = R^{-T} h mod eps).  Bijective. */
int lfft_index_map(lfft_plan_t plan, int which, int64_t* natural_to_grid);

/* ---- point selectors of lfft_points ----------------------------------- */
#define LFFT_POINTS_SAMPLES 0    /* keys g of G(M), points y = M^{-1} g       */
#define LFFT_POINTS_FREQS 1      /* keys h of G(M^T), points M^{-T} h          */

/* Points of one side in NATURAL order (host outputs, m x d row-major each,
 * either may be NULL).  keys: the integer key of every point, g in the
 * Hermite box of M for the pattern P(M), h in the Hermite box of M^T for the
 * generating group G(M^T) (Section 2.2: pattern, generating group).
 * sym_num: the point's symmetric representative times m, i.e. the integer
 * vector t with M^{-1} g = t / m (samples) or M^{-T} h = t / m (frequencies)
 * modulo Z^d, every coordinate reduced into [-m/2, m/2): the representative
 * in the symmetric pattern Lambda(M) cap [-1/2, 1/2)^d of Section 6.2 (the
 * frequency side is what the Dirichlet mask is evaluated on).  Exact
 * (128-bit intermediates).  Errors: ARG (null plan, which not 0 or 1). */
int lfft_points(lfft_plan_t plan, int which, int64_t* keys, int64_t* sym_num);

/* Workspace bytes needed by lfft_forward / lfft_inverse. */
size_t lfft_workspace_size(lfft_plan_t plan);

/* Unitary lattice DFT  out = F(M) in  (Section 2.2, eq. Fouriermatrix):
 *   out_h = m^{-1/2} sum_g in_g exp(-2 pi i h^T M^{-1} g).
 * in: device complex64 [batch][m] in the selected input order (samples);
 * out: device complex64 [batch][m] (frequencies). */
int lfft_forward(lfft_plan_t plan, const void* in, void* out, void* workspace, uint32_t layout,
                 hipStream_t stream);

/* Inverse (= conjugate transpose) of lfft_forward: in are frequencies,
 * out are samples. */
int lfft_inverse(lfft_plan_t plan, const void* in, void* out, void* workspace, uint32_t layout,
                 hipStream_t stream);

/* lfft_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument, and no allocation of any kind.  The intermediate
 * grid between the passes lives in a fixed 64 MiB array of the library on
 * every device that loads it (held until the process ends), so plans whose
 * lfft_workspace_size() exceeds 64 MiB return UNSUPPORTED.  Every call on
 * one device shares that array: calls that overlap in time on one device
 * (different streams, different threads) race and must not be issued.  The
 * first call on a device looks the array's address up once (no allocation).
 * Same arguments otherwise as lfft_forward.  Errors: ARG, STATE,
 * UNSUPPORTED, HIP. */
int lfft_forward_noalloc(lfft_plan_t plan, const void* in, void* out, uint32_t layout,
                         hipStream_t stream);

/* ---- point values <-> orthonormal-translate coefficients --------------- */
#define LFFT_SAMPLES_TO_COEFFS 0
#define LFFT_COEFFS_TO_SAMPLES 1

/* Change of basis in the space V_M of translates of the Dirichlet kernel
 * phi_M (Section 6.2: the samples of a function are turned into its
 * coefficients in the orthonormal translates T(y) phi_M before the wavelet
 * decomposition).  Derived from eq. subspaces-coeffs: the point values
 * s_x = g(2 pi x), x in P(M), of g = sum_y a_y T(y) phi_M are the cyclic
 * convolution of a with phi_M's samples, so
 *   (F(M) s)_h = sqrt(m) 2^{r(h)/2} (F(M) a)_h
 * with r(h) the number of boundary hyperplanes of the cube M^T[-1/2,1/2]^d
 * the class h lies on (the bracket sum of phi_M's coefficients).
 * direction LFFT_SAMPLES_TO_COEFFS: in = s (NATURAL order of G(M)), out = a
 * (same order), or out = F(M) a (NATURAL order of G(M^T)) if fourier != 0;
 * LFFT_COEFFS_TO_SAMPLES: the inverse (in = a, or F(M) a if fourier != 0;
 * out = s).  The bulk factor sqrt(m) is applied in the FFT's last pass, the
 * 2^{-r/2} of the boundary classes by a kernel over those classes only
 * (O(m^{(d-1)/d}) of them).  The first call builds the plan's table of
 * boundary classes (one host scan of G(M^T) and one small device
 * allocation).  workspace: lfft_basis_workspace_size() bytes.  Batch and
 * layout as lfft_forward (NATURAL orders).  Errors: ARG, STATE, NOMEM,
 * HIP. */
size_t lfft_basis_workspace_size(lfft_plan_t plan);
int lfft_basis_change(lfft_plan_t plan, int direction, int fourier, const void* in, void* out,
                      void* workspace, hipStream_t stream);

/* ---- fast wavelet decomposition (Section 5.3) --------------------------- */

/* Plan `levels` steps M_1 = M, N_l = J^{-1} M_l, M_{l+1} = N_l for a
 * dilation J with q = |det J| channels, 2 <= q <= 16 (Section 5.3, steps
 * 1-5 for any |det J|; Section 6.2 Dirichlet wavelets for q = 2), and
 * `batch` signals.  For q > 2 the paper defines no wavelet: the channel
 * matrix of every fiber {k + N^T g_l : g_l in G(J^T)} (g_0 = 0, the other
 * classes in the natural order of the Hermite box of J^T) has first row
 * u = (a(h_l) / sqrt q)_l and the other rows from the reflection
 * I - 2 v v^T / (v^T v), v = u + sign(u_0) e_0 (sign(0) = +1); it is
 * orthogonal when the mask satisfies sum_l a(h_l)^2 = q.  The mask
 * gradients of q > 2 differentiate through the reflection (sign(u_0) held
 * constant on each fiber).  Errors: ARG,
 * SINGULAR, NOT_INTEGRAL, OVERFLOW, UNSUPPORTED (q > 16, d > 4), NOMEM,
 * HIP.  flags: 0, LFFT_HOST_ONLY, LWT_SINGLE_STREAM. */
int lwt_plan_create(lwt_plan_t* plan, int d, const int64_t* M, const int64_t* J, int levels,
                    int64_t batch, uint32_t flags);
int lwt_plan_destroy(lwt_plan_t plan);

/* Level l (0-based) data: N_l (d x d row-major), m_l = |det M_l|, the
 * elementary divisors of N_l (host outputs, any may be NULL). */
int lwt_level_info(lwt_plan_t plan, int level, int64_t* N, int64_t* m_level, int64_t* eps_N);

/* Scaling step of level l (Section 5.2, Theorem 3), for a dilation whose
 * pattern P(J) is cyclic (d_J = 1; UNSUPPORTED otherwise).  Host outputs,
 * any may be NULL: d_M, d_N, the pattern dimensions of M_l and N_l
 * (d_M = d_N + 1: the step adds a cycle; d_M = d_N: it grows one); key[d],
 * the natural sample key in G(M_l) of the step's direction N_l^{-1} z, where
 * z = J^{-1} g and g is the first key of G(J) in the natural order of the
 * Hermite box of J whose class generates G(J) (the direction is a class
 * modulo P(N_l); this representative has key g reduced into the Hermite box
 * of M_l); grid[d], its coordinates Q^{-1} key mod eps in the forward Smith
 * basis of M_l (0 on trivial axes), the basis lfft_index_map uses. */
int lwt_level_scaling(lwt_plan_t plan, int level, int* d_M, int* d_N, int64_t* key, int64_t* grid);

/* Fiber maps of level l (0-based) exactly as the split/unsplit kernels
 * address them (Section 2.2 eq. decomposition applied to
 * G(M_l^T) = G(N_l^T) + N_l^T G(J^T); Section 5.3 steps 2-3), for the natural
 * indices k = k0 .. k0 + count - 1 of G(N_l^T) (host outputs, either may be
 * NULL):
 *  lifts[(k - k0) * q + j]: NATURAL index in G(M_l^T) of the fiber member
 *    k + N_l^T g_j reduced into the Hermite box of M_l^T, g_0 = 0 and, for
 *    q = 2, g_1 = g0 the nonzero class of G(J^T) (so member 1 is the partner
 *    h0 + s, s = N_l^T g0); for q > 2 the classes of G(J^T) in the natural
 *    order of the Hermite box of J^T.  Every class of G(M_l^T) is a member of
 *    exactly one fiber.
 *  phase[k - k0] (q = 2 only; must be NULL for q > 2): the residue rho in
 *    [0, m_l) of the wavelet phase phi(h0) = exp(-2 pi i h0^T M_l^{-1} J y0)
 *    = exp(-2 pi i rho / m_l), y0 the nonzero point of P(J) in
 *    [-1/2, 1/2)^d (Section 6.2 wavelet symbol).
 * path: 0 the kernels' choice for this level, 1 the 32-bit index path
 * (UNSUPPORTED if the level's bounds exclude it), 2 the 64-bit path.
 * Errors: ARG (level, path or range out of bounds), UNSUPPORTED. */
int lwt_fiber_map(lwt_plan_t plan, int level, int path, int64_t k0, int64_t count,
                  int64_t* lifts, int64_t* phase);

/* Coefficient layout of lwt_decompose (host outputs, any may be NULL):
 * q = |det J| channels per level, nblocks = levels (q - 1) + 1 blocks, and per
 * block its element offset and length within one signal's m coefficients,
 * its level (0-based) and channel (1 .. q-1 wavelet channels, 0 for the
 * final low-pass block of the last level).  Arrays hold nblocks entries;
 * call once with NULL arrays to learn nblocks. */
int lwt_coeff_layout(lwt_plan_t plan, int* q, int* nblocks, int64_t* offset, int64_t* length,
                     int* level, int* channel);

/* Dirichlet scaling mask of level l (Section 6.2): host float[m_l] in
 * NATURAL order of G(M_l^T); values sqrt(q) 2^{(r_M - r_N)/2} (the quotient
 * of the Dirichlet kernels' coefficients; 2^{(1 + r_M - r_N)/2} for q = 2) on
 * the closed N_l-box of symmetric representatives, 0 elsewhere. */
int lwt_dirichlet_mask(lwt_plan_t plan, int level, float* mask);

/* Workspace bytes of every lwt_* execute call, and complex64 elements of
 * the `saved` buffer used for differentiation (batch * sum_l m_l). */
size_t lwt_workspace_size(lwt_plan_t plan);
size_t lwt_saved_elems(lwt_plan_t plan);

/* Decomposition (Section 5.3, steps 1-5, levels chained through the
 * low-pass Fourier data): samples [batch][m] NATURAL order of G(M) ->
 * coeffs [batch][m] = [d2^(1) | ... | d2^(L) | d1^(L)], block l in NATURAL
 * order of G(N_l); for q > 2 the blocks of level l are its channels
 * 1 .. q-1 (m_l / q each) and the last block is channel 0 of level L:
 * [lvl 1: ch 1 | .. | ch q-1] .. [lvl L: ch 1 | .. | ch q-1] [ch 0].
 * masks: host array of `levels` device pointers, mask l
 * float[m_l] in NATURAL order of G(M_l^T) (real scaling symbol; the wavelet
 * symbol is derived from it).  saved: NULL or device complex64 buffer of
 * lwt_saved_elems() receiving the per-level Fourier inputs (needed by
 * lwt_decompose_backward for mask gradients; for q > 2 the decomposition
 * then also runs every level's channels one level at a time). */
int lwt_decompose(lwt_plan_t plan, const void* samples, const float* const* masks, void* coeffs,
                  void* saved, void* workspace, hipStream_t stream);

/* Reconstruction (inverse of lwt_decompose; synthesis gamma = sum_j sum_y
 * d_{j,y} T(y) g_j of Section 5.3).  saved: NULL or buffer of
 * lwt_saved_elems() receiving the per-level synthesis inputs (q = 2:
 * d1hat, d2hat; q > 2: channel 0, then channels 1 .. q-1) for
 * lwt_reconstruct_backward. */
int lwt_reconstruct(lwt_plan_t plan, const void* coeffs, const float* const* masks, void* samples,
                    void* saved, void* workspace, hipStream_t stream);

/* Adjoint of lwt_decompose: grad_samples = D^H grad_coeffs, and, if
 * grad_masks (host array of device pointers) is non-NULL, d loss / d mask_l
 * summed over the batch, using `saved` from lwt_decompose (ARG if NULL).
 * Gradients follow the convention G = dL/dRe + i dL/dIm. */
int lwt_decompose_backward(lwt_plan_t plan, const void* grad_coeffs, const void* saved,
                           const float* const* masks, void* grad_samples, float* const* grad_masks,
                           void* workspace, hipStream_t stream);

/* Adjoint of lwt_reconstruct, with mask gradients from its `saved`. */
int lwt_reconstruct_backward(lwt_plan_t plan, const void* grad_samples, const void* saved,
                             const float* const* masks, void* grad_coeffs,
                             float* const* grad_masks, void* workspace, hipStream_t stream);

/* ---- batched transforms on patterns of different M ---------------------- */

/* Many lattices in one call: the signals of lattices M_0 .. M_{count-1}
 * (each d x d, row-major, stored one after another in Ms) are concatenated,
 * signal i holding m_i = |det M_i| complex64 values at element offset
 * offsets[i] = m_0 + ... + m_{i-1}.  Every lattice is transformed
 * independently, natural order in and out, with the unitary transform of
 * lfft_forward / lfft_inverse.  Within one pass the pencils act on disjoint
 * blocks of the data (Section 4.2, the remark after Theorem 2), so the tiles
 * of the same pass of all lattices share one launch.  The plan holds, for the configuration in
 * use, a fixed-tile schedule of every lattice whose elementary divisors are
 * powers of two and 32 <= m_i <= 2^(2 tile_lg); other lattices run through
 * their own lfft plan after the batched launch. */
typedef struct lfft_batch_s* lfft_batch_t;

#define LFFT_BATCH_LOOP 0        /* one lfft launch sequence per lattice      */
#define LFFT_BATCH_PERSISTENT 1  /* two persistent launches over all lattices:
                                    every first pass, then every second pass */
#define LFFT_BATCH_GRAPH 2       /* the persistent launch as a HIP graph,
                                    captured on first use for each (direction,
                                    in, out, workspace) and replayed after    */

/* Create a batch plan (default configuration tile_lg 12, order 0).  flags:
 * 0 or LFFT_HOST_ONLY (schedules only; execute/tune/status return
 * LFFT_E_STATE).  Errors: ARG, SINGULAR, OVERFLOW, UNSUPPORTED (some
 * m_i >= 2^31 or sum m_i >= 2^40), NOMEM, HIP. */
int lfft_batch_create(lfft_batch_t* plan, int count, int d, const int64_t* Ms, uint32_t flags);
int lfft_batch_destroy(lfft_batch_t plan);

/* offsets[count + 1]: element offset of every signal and the total (host). */
int lfft_batch_offsets(lfft_batch_t plan, int64_t* offsets);

/* Workspace bytes of lfft_batch_execute / lfft_batch_tune: 8 * sum m_i,
 * plus one shared region for lattices with a chirp-z axis whose own plan
 * needs more than their slot. */
size_t lfft_batch_workspace_size(lfft_batch_t plan);

/* Select a configuration: tiles of 2^tile_lg elements (11, 12 or 13) and
 * order bits (bit 0: strided pass first when there is no four-step split;
 * bit 1: smallest radix first inside a digit; bit 2: split the pass
 * boundary inside an axis even where an axis boundary fits).  Rebuilds the
 * schedules and the device queues; drops captured graphs.  Errors: ARG. */
int lfft_batch_configure(lfft_batch_t plan, int tile_lg, int order);

/* Configuration in use and the number of lattices it schedules in the
 * batched launch (host outputs, any may be NULL). */
int lfft_batch_config(lfft_batch_t plan, int* tile_lg, int* order, int* eligible);

/* Fixed-tile schedule of lattice i (forward): number of passes (0 if the
 * lattice is not in the batched launch), and per pass (at most 2) the
 * pencil length, the number of tiles and whether the four-step twiddle
 * follows it (host outputs). */
int lfft_batch_schedule(lfft_batch_t plan, int i, int* passes, int64_t* pencil, int64_t* tiles,
                        int* post);

/* Autotuner: time every candidate configuration (tile_lg in {11, 12, 13},
 * order in {0, 1, 2, 3}) with the persistent launch on the caller's buffers
 * (reps timed runs each, minimum kept), keep the fastest, and remember it
 * for this process keyed by the device architecture, the plan flags and
 * the list of matrices: a later call with the same key applies the
 * remembered choice without timing (*best_ms = -1).  Overwrites out and the
 * workspace.  Synchronises. */
int lfft_batch_tune(lfft_batch_t plan, const void* in, void* out, void* workspace, int reps,
                    float* best_ms, hipStream_t stream);

/* The tuner's choices on disk, so that they survive the process.  Every
 * choice is remembered under the device architecture it was timed on (e.g.
 * "gfx950", without feature suffixes), the plan flags and the exact list of
 * matrices.  lfft_batch_tune_save writes every choice this process holds
 * (tuned or loaded) to `path` as JSON:
 *   {"format": "lfft-batch-tune", "version": 1, "entries": [
 *     {"arch": "gfx950", "d": 2, "flags": 0, "matrices": [row-major, every
 *      lattice's d x d matrix concatenated], "tile_lg": 13, "order": 3,
 *      "ms": 0.455}, ...]}
 * (ms: the tuned time, -1 if unknown).  Errors: ARG (null or empty path),
 * IO (cannot write). */
int lfft_batch_tune_save(const char* path);

/* Merge the entries of a file written by lfft_batch_tune_save whose arch
 * equals `arch` (NULL: the current device's architecture) into this
 * process's choices, replacing choices with the same key; lfft_batch_tune on
 * those matrices and flags then applies them without timing.  The whole file
 * is validated first: a malformed file changes nothing.  *loaded (may be
 * NULL) receives the number of entries taken.  Errors: ARG (null or empty
 * path), IO (cannot read, or not such a file), HIP (arch NULL and no
 * device). */
int lfft_batch_tune_load(const char* path, const char* arch, int* loaded);

/* Forget every remembered choice of this process; *count (may be NULL)
 * receives how many there were. */
int lfft_batch_tune_clear(int* count);

/* out = F(M_i) in (inverse != 0: F(M_i)^{-1}) for every lattice, in device
 * complex64 [sum m_i], out of place, on `stream`.  mode: LFFT_BATCH_*.
 * Calls on one plan must not overlap in time (they share the queue heads).
 * Errors: ARG, STATE (host-only plan), HIP. */
int lfft_batch_execute(lfft_batch_t plan, int inverse, int mode, const void* in, void* out,
                       void* workspace, hipStream_t stream);

/* ---- per-launch kernel timing (tracing) -------------------------------- */

/* Start recording every kernel this library launches from now on (process
 * wide): two HIP events on the launch stream around each launch, the kernel
 * name and two byte counts of the launch.  Method bytes: the launch's share
 * of the least the operation must move to or from HBM (a lattice FFT moves
 * each complex point once in and once out, 16 B per point, and each of its np
 * passes is credited 16 / np B per point; a split level 20 B per point, 4 of
 * them the mask).  Pass bytes: the least the launch itself must move (16 B per
 * point for every FFT pass; the method bytes for every other kernel).
 * capacity: maximum number of launches kept. */
int lfft_trace_begin(int capacity);
/* Stop recording; *count receives the number of recorded launches. */
int lfft_trace_end(int* count);
/* Launch i of the last trace (host outputs, any may be NULL): kernel name
 * (static string), method bytes, pass bytes and duration in ms (waits for the
 * launch to complete). */
int lfft_trace_get(int i, const char** name, double* bytes, double* pass_bytes, float* ms);

/* Static description of a status code. */
const char* lfft_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* LFFT_H */
