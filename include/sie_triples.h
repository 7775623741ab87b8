/*
 * sie_triples.h -- C ABI of the MI355X (gfx950) per-fragment (T) library.
 *
 * What it computes: the closed-shell in-situ perturbative-triples energy E_x of
 * one embedded SIE cluster (the paper's section "The In-situ Form of
 * Perturbative (T) in SIE", equation E_corr_CCSD_T with the W, V, D, P and R
 * definitions printed after it), and the sum E = sum_x E_x over clusters
 * (equation C_f of the same section), from
 *   orbital energies e_i, e_a           (canonical cluster orbitals),
 *   CCSD amplitudes t_i^a, t_ij^ab,
 *   ERI blocks (ia|bc), (jl|ia), (ia|jb) in chemists' notation.
 * Readings of the printed equations: the two dummy indices of the W bracket
 * are swapped back to  X = sum_d (ia|bd) t_kj^cd - sum_l (ia|jl) t_lk^bc,
 * and the second term of R is read as the cyclic permutation X_kij.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Layouts are row-major and contiguous, indices i,j,k,l occupied (n_occ),
 * a,b,c,d virtual (n_vir):
 *   eps_occ [n_occ]                      e_i      HOST memory, float64
 *   eps_vir [n_vir]                      e_a      HOST memory, float64
 *   t1      [n_occ][n_vir]               t_i^a    device
 *   t2      [n_occ][n_occ][n_vir][n_vir] t_ij^ab  device, must satisfy t_ij^ab = t_ji^ba
 *   ovvv    [n_occ][n_vir][n_vir][n_vir] (ia|bc)  device, symmetric in b <-> c
 *   ooov    [n_occ][n_occ][n_occ][n_vir] (jl|ia)  device, symmetric in j <-> l
 *   ovov    [n_occ][n_vir][n_occ][n_vir] (ia|jb)  device, symmetric in (ia) <-> (jb)
 * The library reads whichever twin of a symmetric pair suits its access
 * pattern, so inputs that break these symmetries give implementation-defined
 * results.
 * Element type of t1, t2 and the ERI blocks: float64 for SIE_FP64, float32 for
 * SIE_SPLIT_BF16.  Energies are always float64.
 * The orbital energies are host arrays so that every argument check, the
 * requirement max e_occ < min e_vir (every triples denominator D negative)
 * included, runs on the host before any device work.
 *
 * Ownership: the caller owns every buffer (inputs, outputs, workspace); the
 * library keeps no device memory between calls and allocates none.  It owns a
 * few page-locked host buffers (allocated on first use, grown as needed, kept
 * until the process ends) through which it uploads each call's small tables.
 * The host arrays (eps_*, the descriptor structs) may be released when the
 * call returns.
 * Streams: `stream` is a hipStream_t (NULL = the default stream); all device
 * work, the table uploads included, is enqueued on it and the call returns
 * without waiting for the device.  The host waits only when more than four
 * calls' uploads are still queued, and when the finite check is on (see
 * sie_set_check_finite).  A workspace must not be used by two calls that may
 * run at the same time (different streams without ordering between them).
 * Errors: every entry point returns a sie_status; nothing is thrown across
 * the ABI and nothing aborts.  All argument checks run on the host before any
 * HIP call, so a bad argument is reported without touching the device.
 * sie_last_error() gives a message for the last failing call on the calling
 * thread.  On an error no device work has been enqueued unless the status is
 * SIE_ERR_HIP (a launch or copy failed part way; outputs are then undefined).
 */
#ifndef SIE_TRIPLES_H
#define SIE_TRIPLES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIE_ABI_VERSION 2

typedef enum {
  SIE_OK = 0,
  SIE_ERR_INVALID_ARG = 1,   /* bad pointer, size, alignment or orbital energies */
  SIE_ERR_UNSUPPORTED = 2,   /* valid request that this build does not implement */
  SIE_ERR_WORKSPACE = 3,     /* workspace missing or smaller than required        */
  SIE_ERR_NONFINITE = 4,     /* a non-finite orbital energy, or (finite check on)
                                a NaN or infinity in t1, t2 or an ERI block       */
  SIE_ERR_HIP = 5            /* a HIP runtime call failed; see sie_last_error()   */
} sie_status;

typedef enum {
  SIE_FP64 = 0,        /* float64 inputs, float64 contractions and sums          */
  SIE_SPLIT_BF16 = 1   /* float32 inputs split into bf16 hi + lo, three bf16
                          products per contraction with float32 accumulation;
                          denominators and energy sums in float64                */
} sie_precision;

/* One fragment (embedded cluster).  Pointers as described above. */
typedef struct {
  int32_t n_occ;             /* 1 <= n_occ <= SIE_MAX_OCC                      */
  int32_t n_vir;             /* 1 <= n_vir <= SIE_MAX_VIR                      */
  const double* eps_occ;     /* host [n_occ]                                   */
  const double* eps_vir;     /* host [n_vir]                                   */
  const void* t1;            /* device, see layouts                            */
  const void* t2;
  const void* ovvv;
  const void* ooov;
  const void* ovov;
  const double* frag_proj;   /* host [n_occ][n_occ]: the fragment projector C^f_ii'
                                of the same section (in the cluster's occupied
                                orbitals), or NULL for the identity; used by
                                sie_triples_energy and
                                sie_triples_projector_matrix, rejected with
                                SIE_ERR_UNSUPPORTED by the batched and backward
                                entry points                                  */
} sie_fragment;

#define SIE_MAX_OCC 256
#define SIE_MAX_VIR 2048
/* Also s (n_occ^2 n_vir^2 + n_vir^3 + n_vir^2) < 2^32 with s the element size
 * (8 for SIE_FP64, 4 for SIE_SPLIT_BF16): the kernels address each operand
 * with 32-bit byte offsets (40 occupied and 400 virtuals fit in float64);
 * larger fragments get SIE_ERR_UNSUPPORTED. */

/* Gradient outputs of one fragment for sie_triples_backward: device float64
 * arrays with the shapes of the inputs of the same name, or NULL to skip that
 * input's gradient.  eps_occ [n_occ] and eps_vir [n_vir] receive the
 * derivative with respect to the orbital energies (which enter through the
 * triples denominators D only: the diagonal of the canonical cluster Fock
 * matrix), device arrays although the orbital energies themselves are host
 * inputs. */
typedef struct {
  double* t1;
  double* t2;
  double* ovvv;
  double* ooov;
  double* ovov;
  double* eps_occ;
  double* eps_vir;
} sie_fragment_grad;

/* Number of unordered occupied triples i >= j >= k of a fragment:
 * n_occ (n_occ + 1) (n_occ + 2) / 6.  Per-triple outputs are indexed by
 * u = i (i+1) (i+2) / 6 + j (j+1) / 2 + k. */
int64_t sie_occupied_triples(int32_t n_occ);

/* Workspace bytes the energy entry points need for the `n` fragments
 * frags[0..n-1] (host array) at precision `p`, given that at most `max_bytes`
 * may be used (0 = the library's default cap of 16 GiB, or the value of the
 * environment variable SIE_MAX_WORKSPACE_BYTES).  Beyond a fixed part (tables,
 * per-triple partial sums and, for SIE_SPLIT_BF16, the bf16 hi/lo copies of
 * the float32 inputs) the workspace holds the W-tilde cubes of as many
 * occupied triples as fit; a larger workspace means fewer launches.  Returns 0
 * if the arguments are invalid or the minimum exceeds the cap (see
 * sie_last_error()). */
size_t sie_triples_workspace_size(const sie_fragment* frags, int32_t n,
                                  sie_precision p, size_t max_bytes);

/* E_x of one fragment (equation E_corr_CCSD_T).
 *   frag     host pointer to one descriptor
 *   e_out    device float64 [1]: receives E_x
 *   e_triples  device float64 [sie_occupied_triples(n_occ)] or NULL: receives
 *            the contribution of each unordered occupied triple {i, j, k}
 *            (their sum is E_x)
 *   ws       device workspace of ws_bytes >= sie_triples_workspace_size(frag,
 *            1, p, cap) for some cap; its contents on entry are ignored
 * Deterministic: the same inputs give bitwise the same outputs.  The call
 * enqueues the upload of its small tables (fragment descriptors, orbital
 * energies, work list) and its kernels on `stream` and returns. */
sie_status sie_triples_energy(const sie_fragment* frag, sie_precision p,
                              double* e_out, double* e_triples,
                              void* ws, size_t ws_bytes, void* stream);

/* Fragment projector (the C^f factor of equation E_corr_CCSD_T).  The
 * printed sum over a >= b >= c applies C^f to the occupied index paired with
 * one virtual of the sorted triple, which makes the result depend on the
 * order of the virtual orbitals; this library takes the order-independent
 * reading with C acting on the first occupied index of W-tilde:
 *   E_x(C) = (1/3) sum_{ijk abc} (C Wt)_{ijk} R[Wt + Vt]_{ijk} / D_{ijk}
 *          = sum_{i i'} C_{i i'} M_{i i'},
 *   M_{i i'} = (1/3) sum_{jk abc} Wt^{abc}_{i'jk} (R[Wt + Vt] / D)^{abc}_{ijk},
 * which equals the unprojected energy for C = I (tr M = E_x) and is linear
 * in C, so the energies of a complete set of projectors add up to it.
 * sie_triples_projector_matrix writes M (device float64 [n_occ][n_occ],
 * row i, column i'), from which E_x of any projector is a trace; the energy
 * entry point with frag_proj set computes M in its workspace and writes
 * sum C M to e_out (e_triples must then be NULL).  Cost: about three times
 * the energy's (every ordered occupied triple is built: W-tilde and R/D of
 * triples that share two occupied indices are paired).  The workspace of
 * either call is sie_triples_projector_workspace_size (for the energy entry
 * point also what sie_triples_workspace_size returns for a fragment with
 * frag_proj set); frag_proj, when given, must be finite. */
size_t sie_triples_projector_workspace_size(const sie_fragment* frag, sie_precision p,
                                            size_t max_bytes);
sie_status sie_triples_projector_matrix(const sie_fragment* frag, sie_precision p,
                                        double* m_out, void* ws, size_t ws_bytes, void* stream);

/* E_x of one fragment exactly as sie_triples_energy computes it, for callers
 * that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): in place of a caller
 * workspace the call uses a scratch array of SIE_STATIC_SCRATCH_BYTES that
 * the library holds in each GPU's memory from its load on that GPU until the
 * process ends, and it allocates nothing (no device, page-locked or torch
 * memory; its small tables are copied from host memory with pageable copies,
 * which return once the host data has been consumed).  The caller passes the
 * inputs and outputs as for sie_triples_energy.
 *   Limit: the fragment's minimum workspace (sie_triples_workspace_size with
 *   max_bytes = SIE_STATIC_SCRATCH_BYTES) must fit in the scratch, else the
 *   call returns SIE_ERR_WORKSPACE and enqueues nothing.  Fragments that fit
 *   with few triples in flight run in many small rounds.
 *   Concurrency: every call on one GPU shares that GPU's scratch, which keeps
 *   the last call's contents (the call needs none of them).  Two calls on one
 *   GPU that may run at the same time (different streams without ordering,
 *   or different threads) race on the scratch and give undefined results;
 *   calls on one stream are ordered and safe.
 * Results are bitwise equal to sie_triples_energy's for the same inputs. */
#define SIE_STATIC_SCRATCH_BYTES (256u * 1024u * 1024u)
sie_status sie_triples_energy_static(const sie_fragment* frag, sie_precision p,
                                     double* e_out, double* e_triples, void* stream);

/* E_x of each of n fragments and E = sum_x E_x (equation C_f), in one
 * evaluation: the occupied triples of all fragments form one work list,
 * ordered longest first, run in as few launches as the workspace allows.
 *   frags    host array of n >= 1 descriptors, same rules as above
 *   e_frag   device float64 [n]: E_x per fragment
 *   e_total  device float64 [1] or NULL: the sum over fragments
 *   ws       >= sie_triples_workspace_size(frags, n, p, cap) bytes
 * E_x equals what sie_triples_energy gives for the fragment alone (bitwise:
 * the per-fragment reductions run in the same fixed order).  Deterministic;
 * same stream behaviour as sie_triples_energy. */
sie_status sie_triples_energy_batched(const sie_fragment* frags, int32_t n,
                                      sie_precision p, double* e_frag,
                                      double* e_total, void* ws, size_t ws_bytes,
                                      void* stream);

/* Workspace bytes sie_triples_backward needs for the n fragments frags[0..n-1]
 * (host array), with the same cap rule as sie_triples_workspace_size; the
 * backward workspace also holds its contraction lists.  Returns 0 if the
 * arguments are invalid or the minimum exceeds the cap. */
size_t sie_triples_backward_workspace_size(const sie_fragment* frags, int32_t n,
                                           sie_precision p, size_t max_bytes);

/* Gradient of E_x (same equation and readings as sie_triples_energy, C^f =
 * identity) with respect to t1, t2, ovvv, ooov and ovov of each of n
 * fragments.  The energy is not printed as differentiated in the paper; the
 * gradient is the exact adjoint of the energy as computed here: with
 * G = w (R'[Wt] + R'[Wt + Vt]) / D and H = w R'[Wt] / D per occupied triple
 * (w = 2 A_ijk, R' the virtual-index form of R), every contraction that builds
 * Wt is transposed against G and every V-tilde product against H.  Wt is
 * recomputed, not stored.
 *   frags    host array of n >= 1 descriptors (as for the energy).  With
 *            SIE_SPLIT_BF16 Wt is rebuilt from the bf16 hi/lo products, G and
 *            H are held in float32 and the transposed contractions run in
 *            float64 on the float32 inputs; gradients are float64 either way
 *   grad_e   device float64 [n], the upstream derivative dL/dE_x, or NULL
 *            for all ones
 *   grads    host array [n]; each non-NULL pointer is OVERWRITTEN with
 *            grad_e[x] * dE_x / d(input), symmetrized over the input's
 *            index-symmetry orbit (the mean over t_ij^ab and t_ji^ba, over
 *            (ia|bc) and (ia|cb), over (jl|ia) and (lj|ia), over (ia|jb) and
 *            (jb|ia)), so the result does not depend on which twin the
 *            kernels read.  Gradient arrays must not overlap the inputs.
 *            The orbital-energy gradients: dE_x/de_p = sum over the terms of
 *            dE_x/dD times the number of times p occurs in D (+ for
 *            occupied, - for virtual indices); they sum to zero over all
 *            orbitals and satisfy sum_p e_p dE_x/de_p = -E_x.
 *   e_frag   device float64 [n] or NULL: receives E_x
 *   ws       >= sie_triples_backward_workspace_size(frags, n, p, cap) bytes
 * Deterministic (fixed summation order, no atomics); same stream behaviour as
 * sie_triples_energy.  Cost about three times the energy's. */
sie_status sie_triples_backward(const sie_fragment* frags, int32_t n, sie_precision p,
                                const double* grad_e, const sie_fragment_grad* grads,
                                double* e_frag, void* ws, size_t ws_bytes, void* stream);

/* E_x of one fragment given its density-fitting factors in place of the
 * integral blocks.  The paper's in-situ (T) section closes on memory: the
 * method never stores six-index quantities and stays within the CCSD
 * footprint; of the (T) inputs the (ia|bc) block, n_occ n_vir^3 elements, is
 * by far the largest.  Here the caller passes the factors b with
 * (pq|rs) = sum_P b[P][p][q] b[P][r][s], and the library forms (ia|bc),
 * (jl|ia) and (ia|jb) itself on the float64 matrix cores (fixed summation
 * order over P, float64).  With SIE_SPLIT_BF16, (ia|bc) is formed one
 * occupied slice i at a time into a slice buffer, rounded to float32 and
 * split straight into the bf16 hi/lo copies the build reads, so no float32
 * (ia|bc) array exists anywhere; (jl|ia) and (ia|jb) are formed in float32
 * in the workspace.  With SIE_FP64 all three blocks are formed in float64 in
 * the workspace (the same result as sie_triples_energy on the formed blocks;
 * no memory is saved).
 *   frag->b     device float64 [n_aux][n][n], n = n_occ + n_vir, occupied
 *               orbitals first, symmetric in its last two indices (the
 *               formed blocks then have the twin symmetries exactly)
 *   frag->t1, t2  device, as in sie_fragment, float64 (SIE_FP64) or float32
 *               (SIE_SPLIT_BF16)
 *   ws          >= sie_triples_df_workspace_size(frag, p, cap) bytes: the
 *               formed blocks, then what sie_triples_energy needs
 * The finite check (sie_set_check_finite) scans t1, t2 and b.  Same stream
 * behaviour, determinism and error rules as sie_triples_energy; the per-
 * triple output e_triples works as there. */
typedef struct {
  int32_t n_occ;             /* 1 <= n_occ <= SIE_MAX_OCC                      */
  int32_t n_vir;             /* 1 <= n_vir <= SIE_MAX_VIR                      */
  int32_t n_aux;             /* >= 1                                          */
  const double* eps_occ;     /* host [n_occ]                                   */
  const double* eps_vir;     /* host [n_vir]                                   */
  const void* t1;            /* device [n_occ][n_vir]                          */
  const void* t2;            /* device [n_occ][n_occ][n_vir][n_vir]            */
  const double* b;           /* device float64 [n_aux][n][n]                   */
} sie_fragment_df;

size_t sie_triples_df_workspace_size(const sie_fragment_df* frag, sie_precision p,
                                     size_t max_bytes);
sie_status sie_triples_energy_df(const sie_fragment_df* frag, sie_precision p, double* e_out,
                                 double* e_triples, void* ws, size_t ws_bytes, void* stream);

/* MP2 of one cluster or subspace (the paper's embedding workflow, SI section
 * "Systematically Improvable Quantum Embedding Workflow"): amplitudes
 *   t_ij^ab = -(ia|jb) / (e_a + e_b - e_i - e_j),
 * the energy E = sum_ijab t_ij^ab [2 (ia|jb) - (ib|ja)], and the occupied and
 * virtual blocks of the MP2 one-particle density matrix
 *   gamma_ij = 2 delta_ij - 2 sum_k sum_ab t_ik^ab (2 t_jk^ab - t_jk^ba),
 *   gamma_ab = 2 sum_ij sum_c t_ij^ac (2 t_ij^bc - t_ij^cb)
 * (the occupied-virtual block is zero), with the integrals from
 * density-fitting factors, (ia|jb) = sum_P l_ov[i][a][P] l_ov[j][b][P]. */
typedef struct {
  int32_t n_occ;             /* 1 <= n_occ <= SIE_MAX_OCC                      */
  int32_t n_vir;             /* 1 <= n_vir <= SIE_MAX_VIR                      */
  int32_t n_aux;             /* >= 1                                          */
  const double* eps_occ;     /* host [n_occ]                                   */
  const double* eps_vir;     /* host [n_vir], max(eps_occ) < min(eps_vir)      */
  const double* l_ov;        /* device [n_occ][n_vir][n_aux], float64          */
} sie_mp2_input;

/* Workspace bytes of sie_mp2 (energy partial sums; with want_density the
 * amplitudes, unless the caller stores them, and the partial slices of the
 * density products).  0 for invalid arguments. */
size_t sie_mp2_workspace_size(const sie_mp2_input* in, int32_t want_density);

/* MP2 energy and, optionally, amplitudes and density blocks.
 *   e_out     device float64 [1]: E
 *   t2        device float64 [n_occ][n_occ][n_vir][n_vir] or NULL: t_ij^ab
 *   gamma_oo  device float64 [n_occ][n_occ] or NULL
 *   gamma_vv  device float64 [n_vir][n_vir] or NULL
 *   ws        >= sie_mp2_workspace_size(in, gamma_oo || gamma_vv) bytes
 *             (a caller that passes t2 may use less: the amplitudes are then
 *             kept there)
 * The (ia|jb) products run on the float64 matrix cores, one work-group per
 * occupied pair i >= j and 64 x 64 virtual tile pair, forming (ia|jb) and
 * (ib|ja) together so that the energy needs no second pass; the density
 * blocks are batched products over the stored amplitudes.  Deterministic
 * (fixed-order sums); the orbital energies are uploaded with pageable copies
 * that complete before the call returns; everything else is enqueued on
 * `stream`.  At most 361 occupied orbitals (65535 occupied pairs per
 * launch), else SIE_ERR_UNSUPPORTED. */
sie_status sie_mp2(const sie_mp2_input* in, double* e_out, double* t2, double* gamma_oo,
                   double* gamma_vv, void* ws, size_t ws_bytes, void* stream);

/* Kernel timing (diagnostics).  While enabled on the calling thread, every
 * launch made by the entry points above is bracketed by two HIP events on the
 * launch stream.  sie_profile_collect waits for those events, writes the
 * summed elapsed milliseconds and the launch count per kernel class into
 * ms[SIE_PROF_CLASSES] and launches[SIE_PROF_CLASSES] (host arrays), and
 * clears the record.  Classes: 0 = Wt build, 1 = R/D epilogue,
 * 2 = reductions, 3 = split staging (SIE_SPLIT_BF16 only), 4 = gradient
 * contractions (sie_triples_backward; its G/H kernel counts as class 1).
 * Enabling or disabling also clears the record. */
#define SIE_PROF_CLASSES 5
void sie_profile_enable(int on);
sie_status sie_profile_collect(double* ms, int64_t* launches);

/* Tile shapes of the float64 W-tilde build (autotuning).  The build kernel
 * is compiled for sie_tile_variants() tile shapes; sie_tile_variant_shape
 * writes variant v's shape into shape[8] (host): blocks per wave, 16-wide
 * MFMA row tiles and col tiles per wave, work-groups per CU targeted, the
 * work-group's waves along rows and cols (1, 1: waves along blocks), the
 * number of partial-cube layouts (2, or 3: the terms regrouped so that the
 * per-block operand of every term lies on one MFMA side; the row and col
 * tiles then count the per-block side and the shared side; the gradient
 * always builds with a 2-layout shape, variant 0 in place of a 3-layout
 * one), and the k-steps per K-chunk (2: chunks of 8; 4: chunks of 16).  A
 * fragment's variant is the first table entry whose bound is >= its n_vir
 * (variant 0 past the last).  sie_set_tile_table installs a table of n
 * entries (host arrays: strictly ascending bounds >= 1, valid variants) for
 * the whole process, or the built-in tuned table when n = 0.  Energies do not
 * depend on the variant beyond rounding of the contraction order.  Not to be
 * called while another thread runs an evaluation. */
int32_t sie_tile_variants(void);
sie_status sie_tile_variant_shape(int32_t variant, int32_t* shape);
/* The variant the float64 energy of a fragment with n_vir virtuals builds
 * with under the installed table, or -1 for n_vir < 1. */
int32_t sie_tile_variant_of(int32_t n_vir);
sie_status sie_set_tile_table(int32_t n, const int32_t* nv_max, const int32_t* variant);

/* Tile shapes of the split-precision W-tilde build.  A work-group of shape s
 * computes rows x cols of one block of one layout: 64 x 128, 80 x 320,
 * 112 x 256, 64 x 256 (four waves), 160 x 320 (eight waves) and 160 x 160
 * (four waves) for s = 0 .. 5.
 * sie_split_shape_of returns the shape a fragment with n_vir virtuals builds
 * with (-1 for n_vir < 1): the shape of the first entry of the installed
 * table (the built-in one comes from the autotuner's timings) whose bound is
 * >= n_vir, and past the table, among the shapes whose padded tile area is
 * within 10% of the least, the first in the order 5, 4, 1, 2, 3, 0.
 * sie_set_split_table installs a table of n entries (host arrays: strictly
 * ascending bounds >= 1, shapes in [0, SIE_SPLIT_SHAPES)), or the built-in
 * one for n = 0.
 * sie_set_split_shape forces shape s for every fragment of later evaluations
 * (s = -1 restores the default; SIE_ERR_INVALID_ARG outside [-1,
 * SIE_SPLIT_SHAPES)).  Energies do not depend on the shape beyond rounding of
 * the contraction order.  Not to be called while another thread runs an
 * evaluation. */
#define SIE_SPLIT_SHAPES 6
int32_t sie_split_shape_of(int32_t n_vir);
sie_status sie_set_split_shape(int32_t shape);
sie_status sie_set_split_table(int32_t n, const int32_t* nv_max, const int32_t* shape);

/* Finite check.  When on, every energy and backward call first scans t1, t2,
 * ovvv, ooov and ovov of each fragment on the device, waits for the scan, and
 * returns SIE_ERR_NONFINITE (naming the fragment and the array) before any
 * (T) kernel runs if one holds a NaN or an infinity; with the check off such
 * inputs give non-finite outputs.  Default: off, or on when the environment
 * variable SIE_CHECK_FINITE is set to anything but "0" at the first call.
 * Orbital energies are always checked on the host.  Process-wide. */
void sie_set_check_finite(int on);

const char* sie_last_error(void);
int sie_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SIE_TRIPLES_H */
