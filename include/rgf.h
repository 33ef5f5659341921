/*
 * rgf.h -- C ABI of librgf: recursive Green's function (RGF) conductance of
 * armchair graphene nanoribbons on AMD Instinct MI355X (gfx950).
 *
 * Method: S. Ihnatsenka, Comput. Phys. Commun. 183 (2012) 543
 * (arXiv:1107.5300). Eq. (1) defines the retarded Green's function
 * G = (E - H)^{-1} of the ribbon with both leads folded in as self-energies;
 * Eq. (2) the two-terminal conductance G = (2e^2/h) Tr[Gamma_L G^a Gamma_R G^r];
 * Eqs. (3)-(5) the slice-by-slice Dyson recursion that produces the block of
 * G between the first and the last slice; the method section obtains the
 * lead self-energies at the first and last slice separately (here: Sancho-
 * Rubio decimation, in FP64).
 *
 * Model (model paragraph, Fig. 1(a)): N atoms per transverse slice (one p
 * orbital each) along a zigzag chain, L slices, nearest-neighbour hopping t.
 * Slice i (1..L) couples to slice i+1 through the rows k = 0..N-1 with
 * (k + i + parity) even. On-site energies eps[r][i][k] describe disorder
 * realization r; the two semi-infinite leads are pristine ribbons of the same
 * width. z = E + i*eta is used in the leads and in the device.
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers to float64 data (complex values
 *     never cross the boundary, except the debug export of the lead
 *     self-energies, which is interleaved (re, im) float64), in row-major
 *     C order, owned by the caller. The library allocates no device memory on
 *     any path: scratch space is the caller's workspace (for
 *     rgf_conductance_noalloc, a fixed device array inside the library).
 *   - Calls are asynchronous on the caller's HIP stream (hipStream_t passed as
 *     void*; NULL = the null stream). The return value reports only errors
 *     found before anything is enqueued (invalid arguments, an undersized
 *     workspace, a width the kernels do not support) or a failed launch; on
 *     such an error nothing is written.
 *   - Numerical failures of a (realization, energy) tuple are reported per
 *     tuple in status_out (RGF_TUPLE_*), with T = NaN, without a host sync.
 *   - Energies, t, eta and eps are in eV; conductances in units of 2e^2/h;
 *     gradients in (2e^2/h)/eV.
 *   - Not thread-safe per stream: concurrent calls on one stream are ordered
 *     by the stream; calls on different streams must use different
 *     workspaces.
 */
#ifndef RGF_H
#define RGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RGF_ABI_VERSION_MAJOR 1
#define RGF_ABI_VERSION_MINOR 3

/* Ribbon geometry and model constants. */
typedef struct {
  uint32_t struct_size; /* = sizeof(rgf_ribbon_desc), for versioning        */
  int32_t width_n;      /* N atoms per transverse slice, 2..RGF_MAX_WIDTH    */
  int32_t length_l;     /* L slices in the scattering region, >= 1          */
  int32_t parity;       /* 0 or 1: slice i bonds rows (k + i + parity) even */
  double hopping_ev;    /* t, finite and != 0 (e.g. -2.7)                    */
  double eta_ev;        /* eta > 0 and finite (e.g. 1e-8)                     */
} rgf_ribbon_desc;

#define RGF_MAX_WIDTH 512

/* Widths up to RGF_TILE_MAX_WIDTH keep each half-slice (ceil(N/2) rows) in
 * one workgroup's registers and support every entry point and precision.
 * Wider ribbons (RGF_TILE_MAX_WIDTH < N <= RGF_MAX_WIDTH) keep the
 * half-slice matrices in the workspace (Gauss-Jordan by column panels with
 * partial pivoting over the full height) and support FP64 only: every entry
 * point with RGF_PREC_FP64 (rgf_autotune has nothing to tune); the FP32
 * modes return RGF_ERR_UNSUPPORTED for them. */
#define RGF_TILE_MAX_WIDTH 256

/* Arithmetic of the slice recursion. The lead self-energies, the running
 * propagator G_1i and the trace are FP64 in every mode. */
enum {
  RGF_PREC_FP64 = 0,  /* complex128 throughout                                  */
  RGF_PREC_MIXED = 1, /* complex64 slice inversions + FP64 residual refinement  */
  RGF_PREC_FP32 = 2   /* complex64 slice inversions, no refinement (accuracy
                         study of single precision; not for production)       */
};

enum {
  RGF_OK = 0,
  RGF_ERR_INVALID_ARG = -1,
  RGF_ERR_HIP = -2,
  RGF_ERR_WORKSPACE = -3,
  RGF_ERR_UNSUPPORTED = -4
};

enum {
  RGF_TUPLE_OK = 0,
  RGF_TUPLE_NO_CONVERGENCE = 1, /* lead decimation hit its iteration cap     */
  RGF_TUPLE_SINGULAR = 2,       /* exact zero pivot in a slice inversion     */
  RGF_TUPLE_NONFINITE = 3,      /* T came out NaN or Inf                     */
  RGF_TUPLE_OUT_OF_RANGE = 4,   /* T outside [0, number of lead modes]: the
                                   recursion lost its accuracy             */
  RGF_TUPLE_ILL_CONDITIONED = 5 /* the half-slice recursion (each slice
                                   inverted as its two row classes) is too
                                   ill-conditioned for this tuple: its
                                   summed condition estimates say the
                                   rounding error of T could pass ~1e-9.
                                   Happens for pristine or nearly pristine
                                   ribbons within ~1e-3 eV of E = 0, where
                                   cutting a slice between its row classes
                                   leaves zero-energy dangling-bond states.
                                   rgf_conductance, rgf_conductance_noalloc,
                                   rgf_conductance_batched and
                                   rgf_channel_transmission (FP64 and
                                   mixed) then recompute the tuple with
                                   whole N x N slice inversions and never
                                   return this code; rgf_grad and rgf_ldos
                                   report it with NaN outputs             */
};

/* Bytes of device workspace the call with the same arguments needs.
 * want_grad != 0 sizes it for rgf_grad with checkpoint stride ckpt_stride
 * (0 = automatic). Returns 0 for invalid arguments (see rgf_last_error_message). */
size_t rgf_workspace_bytes(const rgf_ribbon_desc* desc, int64_t n_energies,
                           int64_t n_real, int precision, int want_grad,
                           int64_t ckpt_stride);

/* Conductance T[r][e] (Eq. (2)) for every realization r and energy e.
 *   energies_ev   [n_energies]
 *   onsite_eps_ev [n_real][L][N], or NULL for pristine ribbons (then n_real
 *                 is the number of identical output rows). An entry of
 *                 +inf removes that atom (a vacancy: the site decouples
 *                 from its bonds and the leads, the limit eps -> +inf);
 *                 every entry point accepts it, and the gradient and LDOS
 *                 at a vacancy are 0. Other non-finite entries (NaN,
 *                 -inf) are not supported and are not checked.
 *   T_out         [n_real][n_energies]
 *   status_out    [n_real][n_energies] int32, or NULL
 * The recursion follows Eqs. (4)-(5); the lead self-energies (method
 * section) are computed once per energy and shared by all realizations. */
int rgf_conductance(const rgf_ribbon_desc* desc, const double* energies_ev,
                    int64_t n_energies, const double* onsite_eps_ev,
                    int64_t n_real, int precision, double* T_out,
                    int32_t* status_out, void* workspace,
                    size_t workspace_bytes, void* hip_stream);

/* Conductance split over the incoming channels of the left lead (Eq. (2) in
 * the eigenbasis of Gamma_L): the left lead's P = ceil(N/2) transverse mode
 * chains each carry at most one channel, with broadening d_p = -2 Im sigma_p
 * (sigma_p as returned by rgf_lead_modes), and
 *   T_channel_out[r][e][p] = d_p sum_q d_q |(Phi_L^T G_{1L} Phi_R)_pq|^2,
 * whose sum over p is T_out[r][e] (Phi the mode vectors on the rows that
 * bond to each lead). Closed modes give T_p ~ 0 (of order eta). A pristine
 * ribbon gives T_p = 1 for every open channel.
 *   T_channel_out [n_real][n_energies][P]; T_out, status_out as in
 *   rgf_conductance (status_out may be NULL); T_p = NaN for tuples that are
 *   not RGF_TUPLE_OK. precision must be RGF_PREC_FP64 (else
 *   RGF_ERR_UNSUPPORTED).
 * Workspace: rgf_workspace_bytes(desc, n_energies, n_real, precision, 0, 0). */
int rgf_channel_transmission(const rgf_ribbon_desc* desc, const double* energies_ev,
                             int64_t n_energies, const double* onsite_eps_ev,
                             int64_t n_real, int precision, double* T_channel_out,
                             double* T_out, int32_t* status_out, void* workspace,
                             size_t workspace_bytes, void* hip_stream);

/* Conductance and the gradient of L = sum_{r,e} dL_dT[r][e] * T[r][e] with
 * respect to every on-site energy (vector-Jacobian product of Eq. (2)
 * through Eqs. (1), (4), (5)):
 *   dL_deps[r][i][k] = sum_e dL_dT[r][e] * dT[r][e] / d eps[r][i][k].
 * dL_deps is overwritten. ckpt_stride: half-slices between stored restart
 * states of the forward sweep (0 = automatic, about sqrt(2L)); memory for
 * the backward sweep is O((2L/ckpt_stride + ckpt_stride) N^2) per tuple. */
int rgf_grad(const rgf_ribbon_desc* desc, const double* energies_ev,
             int64_t n_energies, const double* onsite_eps_ev, int64_t n_real,
             int precision, const double* dL_dT, double* T_out,
             double* dL_deps, int64_t ckpt_stride, int32_t* status_out,
             void* workspace, size_t workspace_bytes, void* hip_stream);

/* Local density of states of every device site s = (slice i, row k):
 *   ldos_out[r][e][i][k] = -Im G_ss(E_e) / pi   (states per eV per site),
 * the diagonal of the Green's function of Eq. (1), from Dyson's equation
 * (Eq. (3)) applied backwards over the slices after the forward sweep of
 * Eqs. (4)-(5) (the paper names the charge density among the quantities the
 * Green's function gives; this is its spectral density at energy E).
 *   ldos_out [n_real][n_energies][L][N]
 *   T_out    [n_real][n_energies], or NULL
 *   status_out [n_real][n_energies] int32, or NULL; a tuple that is not
 *              RGF_TUPLE_OK gets NaN in all of its L*N entries.
 * The workspace is the one rgf_grad uses: rgf_workspace_bytes(desc,
 * n_energies, n_real, precision, want_grad = 1, ckpt_stride). */
int rgf_ldos(const rgf_ribbon_desc* desc, const double* energies_ev,
             int64_t n_energies, const double* onsite_eps_ev, int64_t n_real,
             int precision, double* ldos_out, double* T_out, int64_t ckpt_stride,
             int32_t* status_out, void* workspace, size_t workspace_bytes,
             void* hip_stream);

/* Conductance with the recursion split along the ribbon length (parallel in
 * L), for batches of (realization, energy) tuples too small to fill the
 * GPU. The paper remarks that parallelising the calculation needs a
 * modification of the recursion of Eqs. (4)-(5); here each tuple's L slices
 * are cut into G segments of consecutive slices, each closed at both ends by
 * the self-energy of a semi-infinite pristine ribbon (the leads' own at the
 * ribbon's ends). Every segment is solved on its own by the left-connected
 * sweep (corners G[a, b], G[b, b]) and, for all but the first, the same
 * sweep over the reversed segment (corner G[a, a]), each on a workgroup of
 * its own; the segments are then joined pairwise in a tree of ceil(log2 G)
 * levels by Dyson's equation (Eq. (3)) across the inter-slice bonds, which
 * also takes the closing self-energies out again.
 * The result is T of Eq. (2) as from rgf_conductance (equal up to rounding);
 * the work is about 1.7x that of one sweep, spread over up to (2G - 1)
 * workgroups per tuple.
 *   n_segments   G; 0 picks the largest G whose n_tuples (2G - 1) workgroup
 *                items run at once, with at least two slices per segment;
 *                G = 1 when the tuples alone fill the GPU. Clamped to
 *                [1, min(L, 1024)]
 *   segments_out (may be NULL) receives the G used
 * Other arguments as for rgf_conductance, FP64 only, widths up to
 * RGF_TILE_MAX_WIDTH (RGF_ERR_UNSUPPORTED above). Tuples the accuracy guard
 * rejects are recomputed by the whole-slice sweep, as in rgf_conductance.
 * The workspace is rgf_segments_workspace_bytes(desc, n_energies, n_real,
 * n_segments) bytes: per tuple and segment three ceil(N/2)^2 complex128
 * matrices (padded to the tile), eight more per joining workgroup, the lead
 * tables and a reversed copy of the on-site energies. */
size_t rgf_segments_workspace_bytes(const rgf_ribbon_desc* desc, int64_t n_energies,
                                    int64_t n_real, int32_t n_segments);
int rgf_conductance_segments(const rgf_ribbon_desc* desc, const double* energies_ev,
                             int64_t n_energies, const double* onsite_eps_ev, int64_t n_real,
                             int32_t n_segments, double* T_out, int32_t* status_out,
                             int32_t* segments_out, void* workspace, size_t workspace_bytes,
                             void* hip_stream);

/* Several ribbons of different widths in one call (energy sweeps x disorder
 * realizations x widths). Ribbon d uses descs[d], its on-site energies at
 * onsite_eps_ev + eps_offsets[d] ([n_real][L_d][N_d]) and writes
 * T_out + T_offsets[d] ([n_real][n_energies]) and the same offset into
 * status_out (may be NULL). All ribbons share energies_ev, n_real and
 * precision. When every ribbon has at least as many tuples as the GPU has
 * persistent workgroup slots for it, the ribbons run one after another on
 * hip_stream (costliest first), each on the whole GPU, in one shared
 * workspace. Otherwise they run concurrently: each gets its own part of the
 * workspace and a share of the persistent workgroups proportional to its
 * work (n^3 L per tuple, n = ceil(N/2)), and all but the costliest run on
 * library-owned streams (default priority, created once per device) that
 * are forked from hip_stream by an event and joined back to it before the
 * call's work ends, so the call stays stream-ordered and capturable (the
 * streams are created by the first concurrent call on a device, which must
 * not be made under stream capture); the workspace is then the sum of the
 * parts. With one ribbon this is rgf_conductance. */
size_t rgf_batched_workspace_bytes(const rgf_ribbon_desc* descs, int32_t n_desc,
                                   int64_t n_energies, int64_t n_real,
                                   int precision);
int rgf_conductance_batched(const rgf_ribbon_desc* descs, int32_t n_desc,
                            const int64_t* eps_offsets,
                            const int64_t* T_offsets,
                            const double* energies_ev, int64_t n_energies,
                            const double* onsite_eps_ev, int64_t n_real,
                            int precision, double* T_out, int32_t* status_out,
                            void* workspace, size_t workspace_bytes,
                            void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and kernels as rgf_conductance, with no workspace argument.
 * Scratch comes from a fixed device array inside librgf of
 * RGF_NOALLOC_SCRATCH_BYTES per GPU, held from the first call on that GPU
 * until the process ends; the call allocates nothing. When the normal plan
 * does not fit, fewer persistent workgroups run (same results, lower
 * throughput); a call whose lead tables plus one workgroup slot exceed the
 * array returns RGF_ERR_WORKSPACE before anything is enqueued. Nothing in
 * the array must start at zero. Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (different streams, or several
 * host threads) race and must be serialised by the caller. The first call
 * on a device resolves the array's device address (not a stream operation);
 * make it outside stream capture. Arguments as for rgf_conductance. */
#define RGF_NOALLOC_SCRATCH_BYTES ((size_t)192 << 20)
int rgf_conductance_noalloc(const rgf_ribbon_desc* desc, const double* energies_ev,
                            int64_t n_energies, const double* onsite_eps_ev,
                            int64_t n_real, int precision, double* T_out,
                            int32_t* status_out, void* hip_stream);

/* Lead self-energies (method section; Sancho-Rubio decimation in FP64),
 * restricted to the rows that bond to the device:
 *   sigma_l_out [n_energies][nl][nl][2]  on slice-1 rows (k + parity) even,
 *   sigma_r_out [n_energies][nr][nr][2]  on slice-L rows (k + L + parity) even,
 * with nl, nr the sizes of those row sets (returned through nl_out, nr_out;
 * pass NULL outputs to query the sizes only). Interleaved (re, im) float64.
 * lead_status_out [n_energies] int32 (RGF_TUPLE_*), or NULL. */
int rgf_lead_self_energy(const rgf_ribbon_desc* desc, const double* energies_ev,
                         int64_t n_energies, double* sigma_l_out,
                         double* sigma_r_out, int32_t* lead_status_out,
                         int32_t* nl_out, int32_t* nr_out, void* workspace,
                         size_t workspace_bytes, void* hip_stream);

/* Per-mode lead self-energies sigma_p, p = 1..P (P = ceil(N/2) through
 * n_modes_out; both leads present the same mode chains), from which
 * Sigma_L = Phi_L diag(sigma) Phi_L^T:
 *   method 0: Sancho-Rubio decimation (what every sweep uses);
 *   method 1: mode matching: the closed-form retarded root of each mode
 *             chain's surface equation (the Bloch-mode solution the paper's
 *             eigenproblem gives), an independent cross-check.
 *   sigma_modes_out [n_energies][P][2] interleaved (re, im) float64, or NULL;
 *   lead_status_out [n_energies] int32 (RGF_TUPLE_*), or NULL.
 * Pass NULL outputs to query P only. Workspace: rgf_workspace_bytes(desc,
 * n_energies, 1, RGF_PREC_FP64, 0, 0). */
int rgf_lead_modes(const rgf_ribbon_desc* desc, const double* energies_ev,
                   int64_t n_energies, int method, double* sigma_modes_out,
                   int32_t* lead_status_out, int32_t* n_modes_out, void* workspace,
                   size_t workspace_bytes, void* hip_stream);

/* Autotuner for the register tiling of the slice recursion (the batching
 * form of the method: tile shape and tuples in flight per compute unit).
 * Times every candidate tiling that holds this width, and one or two
 * persistent-grid sizes each, on a short synthetic sweep of the same width
 * (pristine ribbon, min(L, 8) slices, one tuple per slot), synchronising the
 * stream, and remembers the fastest for (width class, precision) in this
 * process; later plans for that width class use it, including
 * rgf_workspace_bytes, so tune before sizing workspaces. Thread-safe. Not
 * for use inside stream capture. The workspace must hold
 * rgf_autotune_workspace_bytes(desc, precision) bytes.
 * chosen_out (may be NULL) receives 100000 * mgj + NW * 10000 + S * 1000 +
 * C * 10 + slots per compute unit of the chosen configuration, mgj = 1 for
 * the forward sweep whose half-slice inversions run as a blocked
 * Gauss-Jordan on the matrix cores (8 waves, half-slices of up to 128
 * rows; the default of RGF_PREC_MIXED for 97..128 rows), 0 for the
 * register tilings. */
size_t rgf_autotune_workspace_bytes(const rgf_ribbon_desc* desc, int precision);
int rgf_autotune(const rgf_ribbon_desc* desc, int precision, void* workspace,
                 size_t workspace_bytes, void* hip_stream, int32_t* chosen_out);

/* Diagnostics of the mixed mode (RGF_PREC_MIXED; the accuracy discussion
 * of the paper names single precision as the error source, and the mixed
 * mode inverts each half-slice in FP32, refines the inverse with FP64 Newton
 * steps and re-inverts it in FP64 when they do not converge). Every forward
 * sweep of the conductance entry points in that mode adds to three counters
 * of the current device, kept by the library (no workspace):
 *   counts_out[0]  half-slices inverted in FP32 and refined,
 *   counts_out[1]  Newton updates applied,
 *   counts_out[2]  half-slices re-inverted in FP64.
 * Waits for hip_stream (not for other streams), then copies the counters to
 * the host array counts_out[3]; reset != 0 zeroes them afterwards. Sweeps
 * running concurrently on the device add to the same counters. Not for use
 * inside stream capture. Returns RGF_ERR_INVALID_ARG for a NULL counts_out,
 * RGF_ERR_HIP without a usable device. */
int rgf_refine_stats(uint64_t* counts_out, int reset, void* hip_stream);

/* Static descriptions. rgf_last_error_message is thread-local and describes
 * the last non-OK return of this thread. */
const char* rgf_status_string(int status);
const char* rgf_last_error_message(void);
int rgf_version(int* major, int* minor);

#ifdef __cplusplus
}
#endif

#endif /* RGF_H */
