/*
 * tft.h -- C ABI of the MI355X (gfx950) truncated FFT library.
 *
 * The library computes the truncated Fourier transform (TFT) and its inverse
 * (ITFT) of D. Harvey, "A cache-friendly truncated FFT", in the paper's
 * Bailey-style 2^l1 x 2^l2 row/column order (Sect. 3, Alg. 1; Sect. 4, Alg. 2),
 * the pointwise products between them (Sect. 2), and the two products built on
 * them: Schoenhage-Strassen in Z[x] (Sect. 5.1) and Schoenhage-Nussbaumer in
 * (Z/mZ)[x] (Sect. 5.2).
 *
 * Conventions shared by every entry point
 *   - Every pointer named x, a, b, c, g, h, out is DEVICE memory owned by the
 *     caller.  The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream; a device fault surfaces at a later call or
 *     synchronisation and is reported as TFT_E_DEVICE.
 *   - On any argument error nothing is launched and nothing is written.
 *   - zeta is passed as an exponent s: zeta = theta^s (Sect. 6), with theta
 *     the ring's shift unit (2 in Z/(2^N+1), y in (Z/mZ)[y]/(y^K+1)).
 *   - Reentrant for distinct buffers and streams.  Executing a transform,
 *     a pointwise product or a created plan allocates no device memory:
 *     tft_forward / itft_inverse copy their descriptors into a caller
 *     workspace (tft_transform_workspace gives its size), explicit and batch
 *     plans upload theirs when they are created.  The products zx_mul_ss and
 *     zmx_mul_nussbaumer build, upload and cache the plans of a new shape on
 *     its first call (host work plus hipMalloc of a few KB); later calls with
 *     that shape allocate nothing.
 *
 * Cell arrays (the array x_0..x_{L-1} of Sect. 2, "Algorithms 1 and 2 operate
 * on an array x_0, ..., x_{L-1}")
 *   FERMAT ring Z/(2^N+1), W = N/32 limbs: an array of C cells is C*W uint32
 *     limbs (cell i at limbs [i*W, (i+1)*W), little-endian) followed by C
 *     uint32 "top" words (cell i's top at index C*W + i).  Cell value =
 *     limbs + top * 2^N; canonical cells lie in [0, 2^N] (top = 1 only for
 *     the residue 2^N, with all limbs zero).  Inputs must be canonical;
 *     outputs are canonical.  Total bytes: C * (W+1) * 4.
 *   NEGA ring (Z/mZ)[y]/(y^K+1): an array of C cells is C*K uint64
 *     coefficients (cell i at [i*K, (i+1)*K), coefficient of y^j at j),
 *     each in [0, m).  Total bytes: C * K * 8.
 */
#ifndef TFT_H
#define TFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFT_OK = 0,
    TFT_E_ARG = 1,         /* a size, length or flag violates the stated ranges */
    TFT_E_RING = 2,        /* ring unsupported or theta has no power of the needed order */
    TFT_E_RANGE = 3,       /* an output does not fit in the limbs the caller gave */
    TFT_E_WORKSPACE = 4,   /* workspace pointer NULL or smaller than required */
    TFT_E_DEVICE = 5,      /* a HIP call failed (launch error, fault, no device) */
    TFT_E_UNSUPPORTED = 6  /* valid request outside what this build implements */
} tft_status;

enum { TFT_RING_FERMAT = 1, TFT_RING_NEGA = 2, TFT_RING_PRIME = 3 };
#define TFT_PRIME_P 2013265921u /* 15 * 2^27 + 1 */

/* The coefficient ring R of Sect. 2.
 *   kind = TFT_RING_FERMAT: R = Z/(2^N+1), theta = 2 of order 2N (Sect. 2 example,
 *          Sect. 5.1).  This build needs N = 32*W with W a power of two, 1 <= W <= 4096.
 *   kind = TFT_RING_NEGA:   R = (Z/mZ)[y]/(y^K+1), theta = y of order 2K (Sect. 5.2).
 *          This build needs K a power of two, 2 <= K <= 4096, and m odd, 3 <= m < 2^62.
 *   kind = TFT_RING_PRIME:  R = Z/pZ with the word-size prime p = m = TFT_PRIME_P
 *          (the small-coefficient case, Sect. 6), theta = 31^15 of order 2^27 (31 is
 *          the smallest primitive root mod p).  A cell is one uint32 residue in
 *          [0, p); an array of C cells is C uint32 (4 C bytes).  Inputs must be
 *          canonical.  No other prime in this build.
 * Unused fields must be zero. */
typedef struct {
    uint32_t kind;
    uint32_t N;
    uint32_t K;
    uint32_t reserved;
    uint64_t m;
} tft_ring;

/* Split policy for the Bailey decomposition (Sect. 2: L = L1 L2).
 * top_l1     log2 of L1 at the top level; 0 = the paper's floor(l/2) (Alg. 1, Alg. 2);
 *            TFT_SPLIT_DC = L1 = 2 at every level above the leaf, i.e. van der
 *            Hoeven's divide-and-conquer TFT/ITFT, the special case l1 = 1 that
 *            the paper's introduction names as the order it improves on (Sect. 1).
 * leaf_log2  log2 of the largest sub-transform run inside one workgroup's LDS;
 *            0 = the largest that fits.  A larger value is accepted for planning
 *            (tft_plan_export) but tft_plan_execute then returns TFT_E_UNSUPPORTED.
 *            Below the top level, sub-transforms above the leaf are split with
 *            the columns one leaf (Fermat and negacyclic rings) or into the
 *            fewest leaf passes, as evenly as they allow (Z/pZ, whose one-word
 *            cells make small jobs all overhead).
 *            Every split gives identical outputs. */
typedef struct {
    uint32_t top_l1;
    uint32_t leaf_log2;
} tft_split;
#define TFT_SPLIT_DC 0xFFFFFFFFu

/* Human-readable name of a status code (static string). */
const char *tft_status_string(int status);

/* Text of the last HIP failure seen by this thread ("" if none): the failing
 * call and HIP's error string.  Set whenever an entry point returns TFT_E_DEVICE. */
const char *tft_last_error(void);

/* TFT_OK if the ring is supported by this build (see tft_ring). */
int tft_ring_check(const tft_ring *ring);

/* Bytes of one cell of `ring` (FERMAT: 4*(N/32+1), NEGA: 8*K); 0 if unsupported. */
uint64_t tft_elem_bytes(const tft_ring *ring);

/* Bytes of a cell array with `cells` cells (layout above). 0 if unsupported. */
uint64_t tft_array_bytes(const tft_ring *ring, uint64_t cells);

/* Device workspace bytes that tft_forward (direction 0) or itft_inverse
 * (direction 1) needs for this shape: the transform's pass descriptors (jobs,
 * leaf programs, base cases), a few KB.  Host work only; f is ignored for the
 * TFT.  Same argument errors as the transforms. */
int tft_transform_workspace(const tft_ring *ring, uint32_t direction, uint32_t l, uint64_t s, uint64_t z, uint64_t n,
                            uint32_t f, uint64_t *bytes);

/* TFT(L, zeta, z, n) of Sect. 2 computed in place by Alg. 1 (Sect. 3).
 *   l       transform length L = 2^l, 1 <= l <= 24 (l <= 27 over Z/pZ, where
 *           ord(theta) = 2^27); L must divide ord(theta).
 *   s       zeta = theta^s (any s; taken mod ord(theta)).
 *   z, n    1 <= z <= L, 1 <= n <= L.
 *   x       cell array of capacity L.  Cells [0, z) hold a_0..a_{z-1}; cells
 *           >= z are never read (a_i = 0 there) and may hold anything.
 *   ws      device workspace of ws_bytes >= tft_transform_workspace(...)
 *           bytes, 256-byte aligned; TFT_E_WORKSPACE if NULL or too small.
 *           The descriptors are copied into it on `stream` (an asynchronous
 *           host-to-device copy from library-owned host memory), so it must
 *           not be in use by another call until this one has finished.
 * On return cells [0, n) hold a_hat_0..a_hat_{n-1} of eq. (1); all other
 * cells are clobbered (Sect. 2: every cell may serve as scratch).  Allocates
 * no device memory; the launch sequence may be captured into a hipGraph. */
int tft_forward(const tft_ring *ring, uint32_t l, uint64_t s, uint64_t z, uint64_t n, void *x, void *ws,
                uint64_t ws_bytes, void *stream);

/* ITFT(L, zeta, z, n, f) of Sect. 2 computed in place by Alg. 2 (Sect. 4).
 *   f in {0, 1}; 1 <= z <= L; z >= n; 1 <= n + f <= L.
 *   x       cell array of capacity L: cells [0, n) hold a_hat_0..a_hat_{n-1},
 *           cells [n, z) hold L*a_n..L*a_{z-1}; cells >= z are never read.
 *   ws      device workspace as for tft_forward (direction 1).
 * On return cells [0, n) hold L*a_0..L*a_{n-1} (NOT divided by L) and, if
 * f = 1, cell n holds a_hat_n; every other cell is clobbered.  Allocates no
 * device memory. */
int itft_inverse(const tft_ring *ring, uint32_t l, uint64_t s, uint64_t z, uint64_t n, uint32_t f, void *x, void *ws,
                 uint64_t ws_bytes, void *stream);

/* Self-test of the transform kernel's arithmetic for FERMAT rings with
 * N = 8192 .. 65536: runs `ncases` single base cases of Alg. 1 / Alg. 2 (the
 * L = 2 cases, Sect. 3 and Sect. 4), one wavefront each, as the leaf kernel
 * runs them.  `cases` and `out` are device arrays of records of 4 + 2W uint32
 * (W = N/32): opcode (the numbering of tft_plan_export), exponent e of
 * zeta = 2^e (mod 2N), top word of x0, top word of x1, then the W limbs of x0
 * and of x1 (cells as in the cell-array layout, canonical).  `out` receives
 * the records after the base case.  TFT_E_UNSUPPORTED for other rings. */
int tft_debug_base_cases(const tft_ring *ring, uint32_t ncases, const void *cases, void *out, void *stream);

/* Measurement aid (not part of the paper): issue rate of the integer
 * instructions the pointwise products are made of, from registers only.
 * Launches `blocks` workgroups of 256 threads; each thread runs `iters`
 * iterations over eight independent accumulators of
 *   kind 0: v_add_u32,  kind 1: v_mad_u64_u32,
 *   kind 2: v_mad_u64_u32 + v_addc_co_u32 (one limb multiply-accumulate),
 * after one short untimed launch.  *ms = the timed launch's duration (HIP
 * events on `stream`; waits for it), *lane_ops = blocks*256*iters*8
 * operations of the kind, *clock_hz = the shader clock over workgroup 0's
 * first wave (s_memtime cycles per 100 MHz s_memrealtime tick, times 1e8).
 * TFT_E_ARG for kind > 2, zero sizes or NULL outputs. */
int tft_alu_rate(uint32_t kind, uint32_t blocks, uint32_t iters, float *ms, uint64_t *lane_ops, double *clock_hz,
                 void *stream);

/* Pointwise products (Sect. 2: u_hat_i = g_hat_i h_hat_i, 0 <= i < n):
 *   c_i = a_i * b_i * 2^(-scale_log2) in R for 0 <= i < n.
 * a, b, c are cell arrays of capacity `cap` (n <= cap); c may alias a or b.
 * scale_log2 folds the division by L = 2^l that the ITFT leaves (Sect. 2). */
int pointwise_mul(const tft_ring *ring, uint64_t n, const void *a, const void *b, void *c, uint64_t cap,
                  uint32_t scale_log2, void *stream);

/* Parameters of a Schoenhage-Strassen product; NULL (or all zero) means the defaults.
 *   N      ring Z/(2^N+1); 0 = the smallest supported N that holds a product cell.
 *   l      transform length 2^l; 0 = smallest with 2^l >= cells of g + cells of h - 1.
 *   split  Bailey split policy (top_l1 = leaf_log2 = 0: paper split, largest leaf).
 *   k      coefficients per ring element (0 or 1: one, as in Sect. 5.1).  With k > 1
 *          coefficient e*k+j of an operand sits in slot j (ws limbs, ws = the output
 *          coefficient bound in limbs) of cell e; a product cell holds 2k-1 slots
 *          (N >= 32 (2k-1) ws) and an output coefficient is the sum of two
 *          overlapping slots.  Results are identical for every k.
 *   pad_rows  0: the transforms are truncated at n, the number of product cells.
 *          1: n is rounded up to whole rows of the top split, n' = L2 ceil(n/L2)
 *          with L2 = L/L1 (the zero-padding of Sect. 6): TFT(g), TFT(h) give n'
 *          values, n' pointwise products, ITFT(L, 1, n', n', 0).  The ITFT then
 *          has no partial last row.  Cells n..n'-1 of the product are zero, so
 *          the result is identical.  Other values: TFT_E_ARG.
 *   zeta_exp  TFT(g) and TFT(h) use zeta = theta^s, s = zeta_exp mod 2N, instead of
 *          Sect. 2's zeta = 1, and the ITFT uses zeta^2: by eq. (1) each forward
 *          output j carries zeta^[j], so product j carries zeta^(2[j]), which is
 *          the weighting of TFT(L, zeta^2) of u; the ITFT with zeta^2 then returns
 *          L u exactly, and every value gives the same product.  About 3N/2 moves
 *          operands that fill less than half an element into its empty half at the
 *          first butterflies, which shortens carry runs there. */
typedef struct {
    uint32_t N;
    uint32_t l;
    tft_split split;
    uint32_t k;
    uint32_t pad_rows;
    uint32_t zeta_exp;
} tft_ss_params;

/* Workspace bytes zx_mul_ss needs for these operand shapes and parameters. */
int zx_mul_ss_workspace(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs,
                        const tft_ss_params *params, uint64_t *bytes);

/* Product u = g h in Z[x] by Schoenhage-Strassen over R = Z/(2^N+1) (Sect. 5.1):
 * pack, TFT(g), TFT(h) (Sect. 2, zeta = 1), n = len_g + len_h - 1 pointwise
 * products with 2^-l folded in, ITFT(L, 1, n, n, 0), unpack.
 *   g      len_g coefficients, g_limbs uint32 limbs each (little-endian), non-negative.
 *   h      len_h coefficients, h_limbs limbs each.
 *   out    len_g + len_h - 1 coefficients, out_limbs limbs each.
 * Needs out_limbs*32 >= 32*(g_limbs + h_limbs) + ceil(log2 min(len_g, len_h)),
 * else TFT_E_RANGE.  ws: device workspace of at least zx_mul_ss_workspace bytes. */
int zx_mul_ss(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
              uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *ws,
              uint64_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * serving loops that forbid hipMalloc): zx_mul_ss with the same arguments
 * minus the workspace, run from a static device array of
 * TFT_STATIC_SCRATCH_BYTES bytes that the library holds on every device it
 * runs on until the process ends.  The array takes the product's cell arrays
 * (zx_mul_ss_workspace bytes, rounded up to 256) and the descriptors of its
 * three transforms (a few KB); a request that needs more returns
 * TFT_E_WORKSPACE (tft_last_error names both sizes) before any device work.
 * Allocates no device memory (the first call with a new shape builds its plans
 * on the host).  Every call on one device uses the same array: calls that
 * overlap on a device (two streams, two threads) race and give wrong
 * results; calls in one stream order are safe.  The output equals
 * zx_mul_ss's bit for bit. */
#define TFT_STATIC_SCRATCH_BYTES (32ull << 20)
int zx_mul_ss_static(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
                     uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *stream);

/* Phase times of one zx_mul_ss call, from HIP events recorded on its stream. */
typedef struct {
    float pack_ms, tft_g_ms, tft_h_ms, pointwise_ms, itft_ms, unpack_ms, total_ms;
    float leaf_kernel_ms;    /* summed durations of the transform (leaf) kernel launches */
    uint32_t leaf_launches;  /* leaf kernel launches of the three transforms */
    uint32_t n;              /* product length len_g + len_h - 1 */
    uint32_t l;              /* transform length 2^l used */
    uint32_t N;              /* ring Z/(2^N+1) used */
} tft_ss_timing;

/* zx_mul_ss, also filling *timing; waits for the work to finish before returning.
 * For measurement: the events add a few microseconds per launch. */
int zx_mul_ss_timed(const uint32_t *g, uint64_t len_g, uint32_t g_limbs, const uint32_t *h, uint64_t len_h,
                    uint32_t h_limbs, uint32_t *out, uint32_t out_limbs, const tft_ss_params *params, void *ws,
                    uint64_t ws_bytes, void *stream, tft_ss_timing *timing);

/* Workspace bytes zmx_mul_nussbaumer needs. */
int zmx_mul_nussbaumer_workspace(uint64_t len_g, uint64_t len_h, uint32_t log2K, uint64_t *bytes);

/* Product u = g h in (Z/mZ)[x] by Schoenhage-Nussbaumer (Sect. 5.2): the
 * inputs are cut into pieces of K/2 coefficients placed in the low half of
 * elements of R = (Z/mZ)[y]/(y^K+1), multiplied through TFT/TFT/pointwise
 * negacyclic products/ITFT over R with theta = y, and recombined by adding
 * the overlapping pieces mod m.
 *   g, h   len_g, len_h coefficients (uint64, each < m); m odd, 3 <= m < 2^62.
 *   log2K  K = 2^log2K, 1 <= log2K <= 12; the transform length 2^l is the
 *          smallest power of two >= (pieces of g) + (pieces of h) - 1 and must
 *          not exceed 2K, else TFT_E_ARG.
 *   out    len_g + len_h - 1 coefficients (uint64, in [0, m)). */
int zmx_mul_nussbaumer(const uint64_t *g, uint64_t len_g, const uint64_t *h, uint64_t len_h, uint64_t m,
                       uint32_t log2K, uint64_t *out, void *ws, uint64_t ws_bytes, void *stream);

/* Workspace bytes zpx_mul_ntt needs: two cell arrays of the transform length. */
int zpx_mul_ntt_workspace(uint64_t len_g, uint64_t len_h, uint64_t *bytes);

/* Product u = g h in (Z/pZ)[x], p = TFT_PRIME_P, through TFT(g), TFT(h), n
 * pointwise products and the ITFT over R = Z/pZ (Sect. 2; the small-coefficient
 * case of Sect. 6), n = len_g + len_h - 1, transform length 2^l the smallest
 * power of two >= n, l <= 27 (else TFT_E_ARG).
 *   g, h      len_g, len_h coefficients (uint32, each < p), device memory.
 *   pad_rows  0: transforms truncated at n; 1: n rounded up to whole rows of
 *             the paper's split (L2 = 2^(l - floor(l/2))), Sect. 6's zero-padding
 *             that leaves the ITFT without a partial row.  Same output.
 *   out       n coefficients (uint32, in [0, p)).
 *   ws        zpx_mul_ntt_workspace bytes.
 * The first call with a new shape builds and uploads its plans. */
int zpx_mul_ntt(const uint32_t *g, uint64_t len_g, const uint32_t *h, uint64_t len_h, uint32_t pad_rows,
                uint32_t *out, void *ws, uint64_t ws_bytes, void *stream);

/* ---- batches of independent Z[x] products ---- */

/* One Schoenhage-Strassen product of a batch (device pointers, as in zx_mul_ss). */
typedef struct {
    const uint32_t *g;
    uint64_t len_g;
    uint32_t g_limbs;
    const uint32_t *h;
    uint64_t len_h;
    uint32_t h_limbs;
    uint32_t *out;
    uint32_t out_limbs;
    tft_ss_params params; /* all zero: the defaults of zx_mul_ss */
} tft_zx_request;

typedef struct tft_batch_plan tft_batch_plan;

/* How a batch plan picks each request's parameters (k, N, l, split, padding):
 *   TFT_POLICY_GIVEN  the request's params as given (all zero = the default
 *                     rule of tft_ss_default_params);
 *   TFT_POLICY_RULE   the default rule for every request, params ignored;
 *   TFT_POLICY_MODEL  the candidate (tft_ss_candidates) of smallest time
 *                     predicted by a cost model (tft_mlp_choose_ss). */
enum { TFT_POLICY_GIVEN = 0, TFT_POLICY_RULE = 1, TFT_POLICY_MODEL = 2 };

/* Plan `count` products for execution together.  Requests are grouped by ring
 * size; in each group pass p of every TFT (resp. ITFT) is one kernel launch,
 * and the pointwise products are one launch.  Requests whose arguments are
 * invalid are skipped and reported by tft_batch_plan_status.
 * max_workspace (bytes, 0 = no limit) splits the requests into consecutive
 * chunks run one after another in the same workspace; a request whose own
 * workspace, rounded up to a multiple of 256 bytes, exceeds the limit is
 * skipped with TFT_E_WORKSPACE.  policy is one of TFT_POLICY_*; `model` is
 * required for TFT_POLICY_MODEL and ignored otherwise (TFT_E_ARG).  The
 * request array is copied; its g, h and out pointers are used by every
 * execution of the plan.  With a device present the plan's descriptors are
 * uploaded to the current device (hipMalloc) and a capture stream is made
 * here, so that executions allocate nothing; without one the plan is host
 * data only. */
int tft_batch_plan_create(const tft_zx_request *reqs, uint32_t count, uint64_t max_workspace, int policy,
                          struct tft_mlp *model, tft_batch_plan **plan);

/* The parameters each request was planned with (count entries), after the
 * policy; entries of skipped requests are as the policy left them. */
int tft_batch_plan_params(const tft_batch_plan *plan, tft_ss_params *params);

/* Device workspace bytes the plan needs. */
uint64_t tft_batch_plan_workspace(const tft_batch_plan *plan);

/* Per-request status (count entries): TFT_OK, or why the request was skipped. */
int tft_batch_plan_status(const tft_batch_plan *plan, int *status);

/* Kernel launches of one execution. */
uint32_t tft_batch_plan_launches(const tft_batch_plan *plan);

/* Run every planned product on `stream`, on the device the plan was created
 * on (TFT_E_ARG otherwise).  use_graph = 0: the launches are issued directly.
 * use_graph = 1: the first call (and any call with another workspace pointer)
 * runs the launches and captures them on the plan's own stream into a
 * hipGraph; later calls replay the graph.  No call allocates device memory
 * (the runtime's graph instantiation aside). */
int tft_batch_plan_execute(tft_batch_plan *plan, void *ws, uint64_t ws_bytes, int use_graph, void *stream);

/* Free a batch plan (host data, device descriptors, graph).  NULL is ignored. */
void tft_batch_plan_destroy(tft_batch_plan *plan);

/* ---- choosing the parameters of a product (not part of the paper) ----
 * A candidate fixes the bundling factor k (then N and l are the smallest the
 * product allows) and the top split of Alg. 1/2.  Every candidate gives the
 * same output bits; only the time differs. */

#define TFT_SS_FEATURES 15

/* The candidate set of a product shape, in a fixed order: k = 1, 2, 4, ..., 32
 * (those the ring sizes allow), each with the paper's split and, when the
 * transform needs more than one leaf, a split whose column pass is one leaf;
 * each of these is followed by its whole-row padded form (pad_rows = 1) when
 * padding changes the truncation, and every one of them by its twisted form
 * (zeta_exp = 3N/2).
 * out == NULL: only *count is set.  TFT_E_ARG if cap < *count. */
int tft_ss_candidates(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, tft_ss_params *out,
                      uint32_t cap, uint32_t *count);

/* The fixed default rule: the smallest k whose cell-array footprint is within
 * 5/4 of the smallest footprint over the candidate k, with the paper's split. */
int tft_ss_default_params(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs,
                          tft_ss_params *out);

/* TFT_SS_FEATURES scaled features of (product shape, candidate) read by the
 * cost model: operand lengths and limbs, k, l, ring size, fill n/L (n the
 * transforms' truncation, padded or not), footprint, pointwise limb products,
 * transform pass bytes, leaf passes of a TFT, top split share, leaf passes of
 * the ITFT, whole-row padding (0/1), forward twist (0/1).  Host work only. */
int tft_ss_features(uint64_t len_g, uint32_t g_limbs, uint64_t len_h, uint32_t h_limbs, const tft_ss_params *p,
                    float *feat);

/* Exhaustive timing of ncand candidates on one request (device buffers; its
 * out is written): per candidate one untimed run, then `reps` runs each
 * bracketed by HIP events on `stream`; ms[c] = median.  *best (if not NULL) =
 * index of the smallest time, ties to the smaller index.  ws must hold the
 * largest candidate's zx_mul_ss_workspace. */
int tft_ss_time(const tft_zx_request *req, const tft_ss_params *cands, uint32_t ncand, uint32_t reps, void *ws,
                uint64_t ws_bytes, void *stream, float *ms, uint32_t *best);

/* fp32 multilayer perceptron predicting log run time from the features:
 * in_features -> `depth` ReLU layers of `hidden` units -> 1 output.  Forward,
 * backward (mean squared error) and Adam run as HIP kernels.  Parameters are
 * one float array: per layer the weights (out x in, row-major) then the
 * biases; initialised He-uniform from `seed` (SplitMix64), biases zero. */
typedef struct tft_mlp tft_mlp;

int tft_mlp_create(uint32_t in_features, uint32_t hidden, uint32_t depth, uint64_t seed, tft_mlp **mlp);
uint64_t tft_mlp_param_count(const tft_mlp *mlp);
/* Copy the n = tft_mlp_param_count parameters to / from host memory. */
int tft_mlp_get_params(const tft_mlp *mlp, float *host, uint64_t n);
int tft_mlp_set_params(tft_mlp *mlp, const float *host, uint64_t n);
/* y[b] = model(x[b]) for `batch` rows; x (batch x in_features) and y are device buffers. */
int tft_mlp_forward(tft_mlp *mlp, const float *x, uint32_t batch, float *y, void *stream);
/* Gradient of loss = sum_b (model(x_b) - target_b)^2 / (2 batch) with respect to
 * the parameters (device buffer of param_count floats, may be NULL), and the
 * loss (device float, may be NULL).  Device buffers throughout. */
int tft_mlp_gradient(tft_mlp *mlp, const float *x, const float *target, uint32_t batch, float *grad,
                     float *loss, void *stream);
/* `iters` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) at rate lr;
 * *final_loss (host, may be NULL) receives the loss after the last step. */
int tft_mlp_train(tft_mlp *mlp, const float *x, const float *target, uint32_t batch, uint32_t iters, float lr,
                  float *final_loss, void *stream);
void tft_mlp_destroy(tft_mlp *mlp);

/* For every request (host array), evaluate the model on all its candidates
 * and store the candidate of smallest predicted time in reqs[i].params
 * (ties to the earlier candidate). */
int tft_mlp_choose_ss(tft_mlp *mlp, tft_zx_request *reqs, uint32_t count, void *stream);

/* ---- explicit plans: transforms with a chosen split, built ahead of use ---- */

typedef struct tft_plan tft_plan;

/* Build the pass schedule of one transform (direction 0 = TFT, 1 = ITFT) and
 * upload its descriptors to the current device (hipMalloc of a few KB).  With
 * no device present the plan is built on the host only (for tft_plan_export
 * and tft_plan_base_cases).  f is ignored for the TFT. */
int tft_plan_create(const tft_ring *ring, uint32_t direction, uint32_t l, uint64_t s, uint64_t z, uint64_t n,
                    uint32_t f, const tft_split *split, tft_plan **plan);

/* Run a plan in place on cell array x (capacity 2^l) on `stream`.  Allocates
 * nothing on the device the plan was created on; the first execution on
 * another device uploads the descriptors there. */
int tft_plan_execute(tft_plan *plan, void *x, void *stream);

/* Free a plan (host and device descriptors).  NULL is ignored. */
void tft_plan_destroy(tft_plan *plan);

/* Number of base-case (L = 2) executions the plan performs, counting
 * executions that change nothing, as in Theorems 1 and 2. */
uint64_t tft_plan_base_cases(const tft_plan *plan);

/* Serialise the plan's schedule into `buf` (uint64 words) for host-side
 * inspection.  *needed receives the word count; if cap_words is too small
 * nothing is written and TFT_E_ARG is returned.  Layout:
 *   [0] version (1)  [1] passes  [2] jobs  [3] programs  [4] steps  [5] ops
 *   [6] ord(theta)   [7] leaf_log2
 *   passes:   per pass   job_begin, job_count, max_len
 *   jobs:     per job    base, stride, program, s, nload, nstore
 *   programs: per prog   step_begin, step_count, len
 *   steps:    per step   op_begin, op_count
 *   ops:      per op     opcode, i0, i1, alog, b   (exponent = s * 2^alog + b mod ord)
 * Opcodes: 0 none, 1 TFT z=2 n=2, 2 TFT z=1 n=2, 3 TFT z=2 n=1,
 *          4 ITFT n=2, 5 ITFT n=1 f=1 z=2, 6 ITFT n=1 f=1 z=1, 7 ITFT n=1 f=0 z=2,
 *          8 ITFT n=1 f=0 z=1, 9 ITFT n=0 z=2, 10 ITFT n=0 z=1
 * (the base cases of Alg. 1 and Alg. 2, L = 2). */
int tft_plan_export(const tft_plan *plan, uint64_t *buf, uint64_t cap_words, uint64_t *needed);

#ifdef __cplusplus
}
#endif

#endif /* TFT_H */
