/*
 * snc.h -- exact bivariate resultants and integer gcds on one AMD MI355X.
 *
 * The two symbolic operations that the curve and curve-pair analyses of
 * Berberich, Emeliyanenko, Kobel and Sagraloff, "Arrangement Computation for
 * Planar Algebraic Curves", rely on:
 *
 *   res_y(f, g) in Z[x] for f, g in Z[x, y]   -- the projection resultant
 *       R = res(f, f_y, y) (Section 2.1, "Projection Phase") and the
 *       curve-pair resultant R_CD = res(f, g, y) (Section 3);
 *   gcd(a, b) in Z[x]                          -- Yun's square-free
 *       factorisation of R (Section 2.1) and the content of f (Section 2.1).
 *
 * Both follow the modular "divide-conquer-combine" scheme of Section 4
 * ("Symbolic Speedups"): modular and evaluation homomorphisms, independent
 * problems over prime fields, interpolation and Chinese remaindering.
 *
 * Integers.  Every integer array is a sequence of little-endian 32-bit limbs
 * in two's complement with a fixed number of limbs per coefficient
 * (nlimbs >= 1).  An int64 array is exactly nlimbs = 2 (no copy needed).
 *
 * Results.  res_y is returned as the determinant of the Sylvester matrix
 * (content and sign kept): rows 0..n-1 hold f's coefficients f_m .. f_0,
 * rows n..n+m-1 hold g's g_n .. g_0, each row shifted one column right of
 * the row above, m and n the y-degrees over Z[x].  res_y(f, g) = 0 when f = 0
 * or g = 0, and 1 when m = n = 0.  gcd(a, b) is the gcd in Z[x] including
 * the integer content, with a positive leading coefficient; gcd(0, 0) = 0.
 *
 * Memory.  Inputs and outputs are HOST buffers.  Device memory is owned by
 * the caller: each compute call takes a device workspace (d_ws, ws_bytes)
 * whose size the matching *_plan call reports, and a HIP stream (passed as
 * void*, a hipStream_t; NULL = the default stream).  The library never
 * allocates device memory.  A call returns after its result is on the host.
 *
 * Errors.  Every function returns an snc_status; nothing aborts or prints.
 * snc_last_error() gives a message for the last failure on a context.
 *
 * Threads.  One snc_ctx per host thread.  A server (snc_server_*) is
 * internally synchronised and may be used from several threads.
 */
#ifndef SNC_H
#define SNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SNC_OK = 0,
  SNC_EINVAL = -1,    /* invalid argument (NULL pointer, negative size, nlimbs < 1, unsupported degree) */
  SNC_ERANGE = -2,    /* output buffer too small; required deg / nlimbs written back into *out */
  SNC_ENOMEM = -3,    /* workspace (or server pool) smaller than the plan requires */
  SNC_EDEVICE = -4,   /* HIP runtime error; see snc_last_error */
  SNC_EAGAIN = -5,    /* server: request not finished yet */
  SNC_EINTERNAL = -6, /* an internal consistency check failed (a bug) */
  SNC_ENOTSUP = -7    /* the input needs a path this library does not have (the message says which) */
} snc_status;

/* f = sum_{i<=dy} sum_{k<=dx} c_{i,k} x^k y^i, coefficient c_{i,k} at
 * limbs[(i*(dx+1)+k)*nlimbs .. +nlimbs).  dy = -1 denotes f = 0 (limbs may
 * be NULL).  Rows of zeros above the true y-degree are allowed: the y-degree
 * over Z[x] is the highest non-zero row. */
typedef struct {
  const uint32_t* limbs;
  int32_t dy, dx, nlimbs;
} snc_bipoly;

/* a = sum_{i<=deg} c_i x^i, c_i at limbs[i*nlimbs .. +nlimbs).  deg = -1 is
 * the zero polynomial.  As an OUTPUT: on entry deg is the capacity (highest
 * degree that fits) and nlimbs the limb stride of the caller's buffer; on
 * return deg is the degree of the result and nlimbs is unchanged (values are
 * sign-extended to the stride).  On SNC_ERANGE, deg and nlimbs receive the
 * required capacity and stride and nothing else is written. */
typedef struct {
  uint32_t* limbs;
  int32_t deg, nlimbs;
} snc_upoly;

typedef struct {
  int32_t deg_bound;      /* bound on the degree of the result */
  int32_t out_nlimbs;     /* limbs per output coefficient that always suffice */
  int32_t nprimes;        /* number of primes the computation starts with */
  int32_t reserved;
  size_t workspace_bytes; /* device workspace the compute call needs */
} snc_plan;

typedef struct snc_ctx snc_ctx;
typedef struct snc_prepared snc_prepared;
typedef struct snc_server snc_server;

/* Version of this interface (major*10000 + minor*100 + patch). */
int snc_version(void);
const char* snc_status_str(int status);

/* Create a context bound to HIP device `device` (makes it current).  Builds
 * the prime table on the host; does no device allocation. */
int snc_create(int device, snc_ctx** out);
int snc_destroy(snc_ctx* ctx);
const char* snc_last_error(const snc_ctx* ctx);

/* Per-stage timing of the last compute call on this context, measured with
 * HIP events on the call's stream (device stages) or the host clock (host
 * stages) when enabled (off by default).  names, ms and launches receive up
 * to `cap` entries; returns the number of stages recorded.  launches is the
 * number of kernel launches of a device stage (0 for a host stage); for the
 * gcd stages it is the number of primes the stage processed. */
int snc_set_timing(snc_ctx* ctx, int enable);
int snc_get_timing(const snc_ctx* ctx, const char** names, float* ms, int32_t* launches, int cap);

/* Throughput ceiling of one integer operation on this context's device,
 * measured (not a compute call of the method): eight independent chains per
 * lane, sixteen wavefronts per CU, the best of three timed launches.  The
 * modular kernels (Section 4, "Symbolic Speedups": problems over prime
 * fields) are built from these operations, so their roofline is stated
 * against these rates beside the nominal int32 VALU peak.
 *   kind SNC_MB_MONTGOMERY: Montgomery products a*b*2^-32 mod p (p < 2^30);
 *        SNC_MB_MUL_LO:     32-bit low multiplies;
 *        SNC_MB_MAD_U64:    32x32+64-bit multiply-adds.
 * iters: chain steps per lane (>= 1).  d_buf: device scratch of at least
 * 64 * 16 * 4 bytes per CU, caller-owned, overwritten.  On SNC_OK
 * *ops_per_s receives the operations per second over the whole device.
 * Errors: SNC_EINVAL (bad kind, iters or NULL), SNC_ENOMEM (buffer too
 * small), SNC_EDEVICE. */
enum { SNC_MB_MONTGOMERY = 0, SNC_MB_MUL_LO = 1, SNC_MB_MAD_U64 = 2 };
int snc_microbench(snc_ctx* ctx, int kind, int32_t iters, void* d_buf, size_t buf_bytes, void* stream,
                   double* ops_per_s);

/* Autotuner of the evaluation kernel (Section 4, "Symbolic Speedups": the
 * problems over prime fields are distributed over the device).  For each
 * register class of the fused evaluation + elimination kernel (largest
 * y-degree 8, 16, 32, 40, 48, 64) a batch uses, the launch variant is chosen:
 * wpe = minimum wavefronts per SIMD the register allocation is held to
 * (1 = unconstrained .. 4), chunk = 0 for one workgroup per block of 64
 * points or the number of blocks a persistent workgroup takes at a time
 * from a device work counter.  All variants give identical results.
 * snc_set_tuning: mode 0 = no measurements (cached choices, else wpe 1,
 *   chunk 0), 1 = measure the classes not yet tuned on this device (the
 *   default; batched calls only: snc_resultant_y_prepare/_batch), 2 =
 *   measure again.  A measurement times every variant on the class's own
 *   launch and keeps, of those within 5% of the fastest, the one that
 *   spills the fewest bytes per lane (spill traffic slows the kernels that
 *   follow, which a launch timed alone does not show).  Choices are kept
 *   per (class, LDS variant, log2 of the
 *   class's block count) and appended to the cache file
 *   $SNC_TUNE_DIR/eval_elim_<arch>_<CUs>cu_r<rev>.tune (default directory
 *   $HOME/.cache/snc), read by later processes; <rev> is the revision of
 *   the evaluation kernels, so a library with changed kernels tunes again.
 * snc_set_eval_variant: force (wpe, chunk) for every launch of the class
 *   whose largest y-degree is class_cap on this context (wpe 0 clears).
 * snc_get_tuning: the last batched preparation's choice per class used:
 *   info[6 i ..] = class_cap, wpe, chunk, persistent grid, source (0
 *   defaults, 1 measured, 2 cached, 3 forced), variants timed; ms[2 i ..] =
 *   measured time of the chosen and of the default variant (source 1);
 *   *tune_ms = host time the tuning took.  Returns the number of classes. */
int snc_set_tuning(snc_ctx* ctx, int mode);
int snc_set_eval_variant(snc_ctx* ctx, int32_t class_cap, int32_t wpe, int32_t chunk);
int snc_get_tuning(const snc_ctx* ctx, int32_t* info, float* ms, int cap, float* tune_ms);

/* ---- resultant res_y(f, g) in Z[x] --------------------------------------
 * Host-only planning: degree bound D (Sylvester weighted-degree bound),
 * Hadamard-type coefficient bound B, number of primes k with prod p > 2B,
 * output limbs L = ceil((log2 B + 2)/32), device workspace. */
int snc_resultant_y_plan(const snc_bipoly* f, const snc_bipoly* g, snc_plan* out);

/* One resultant: reduce mod k primes -> evaluate at D+1 points and eliminate
 * per (prime, point) -> interpolate per prime -> CRT per coefficient.  The
 * result is exact (not probabilistic).  out: see snc_upoly. */
int snc_resultant_y(snc_ctx* ctx, const snc_bipoly* f, const snc_bipoly* g, void* d_ws,
                    size_t ws_bytes, void* stream, snc_upoly* out);

/* n independent resultants in one submission: every stage runs once over
 * all pairs (one launch per stage and degree class), captured once into a
 * HIP graph per batch shape and replayed.  f, g, out are arrays of n. */
int snc_resultant_y_batch_plan(int32_t n, const snc_bipoly* f, const snc_bipoly* g,
                               snc_plan* out_each /* n entries or NULL */, snc_plan* out_total);
int snc_resultant_y_batch(snc_ctx* ctx, int32_t n, const snc_bipoly* f, const snc_bipoly* g,
                          void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out);

/* Prepared resultants: plan n pairs and upload their inputs into the device
 * workspace once (the workspace must stay valid and untouched until the
 * handle is destroyed); each run then executes only the device pipeline,
 * captured as a HIP graph on the first run and replayed, and writes the n
 * results into out (same conventions as snc_resultant_y_batch).  For callers
 * that keep inputs resident and recompute, and for timing the device path
 * without the input transfer.  A handle belongs to its context's thread. */
int snc_resultant_y_prepare(snc_ctx* ctx, int32_t n, const snc_bipoly* f, const snc_bipoly* g,
                            void* d_ws, size_t ws_bytes, void* stream, snc_prepared** out);
int snc_prepared_run(snc_prepared* prep, void* stream, snc_upoly* out);
int snc_prepared_destroy(snc_prepared* prep);

/* Pipelined runs of a prepared batch, for callers that run it repeatedly and
 * want throughput: snc_prepared_submit enqueues one run of the device
 * pipeline on stream, a device copy of its output block into one of two
 * staging slots in d_stage (caller-owned device memory of at least
 * snc_prepared_stage_bytes(prep) bytes, 0 for a batch of trivial pairs; it
 * must stay valid until every submitted run is collected), and the download
 * of that slot to pinned host memory on a second stream of the context; it
 * returns at once with a ticket (0, 1, 2, ... per handle).  The next
 * submit's kernels start right after the copy, while the previous run's
 * results travel.  snc_prepared_collect waits for the ticket's download and
 * writes its n results into out (conventions of snc_prepared_run;
 * SNC_ERANGE leaves the run outstanding).  At most two runs are
 * outstanding: a third submit gives SNC_EAGAIN until one is collected;
 * collecting a ticket that is not outstanding gives SNC_EINVAL; a staging
 * buffer smaller than needed gives SNC_ENOMEM with the sizes in the message.
 * Every run of a handle (submitted or snc_prepared_run) goes to one stream:
 * runs share the workspace and are ordered by that stream only.  The pinned
 * host slots are allocated on the first submit and freed with the handle,
 * which first waits for any uncollected download. */
size_t snc_prepared_stage_bytes(const snc_prepared* prep);
int snc_prepared_submit(snc_prepared* prep, void* d_stage, size_t stage_bytes, void* stream, int64_t* ticket);
int snc_prepared_collect(snc_prepared* prep, int64_t ticket, snc_upoly* out);

/* One resultant with no allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the computation of snc_resultant_y with its device workspace
 * in a fixed module array of SNC_NOALLOC_SCRATCH_BYTES per device (held from
 * the library's first use on the device until the process ends), its upload
 * block in a fixed host array, and the results downloaded into out.  The
 * call makes no device or pinned-host allocation and creates no stream,
 * event or graph (host-side planning uses a few small heap vectors, as every
 * call does).  Arguments and results as for snc_resultant_y.  Errors: a pair
 * whose plan needs more than SNC_NOALLOC_SCRATCH_BYTES (its workspace_bytes
 * from snc_resultant_y_plan) gives SNC_ENOMEM before any device work, with
 * the sizes in the message; SNC_ERANGE as for snc_resultant_y.  Every call
 * on a device shares that device's array: calls that overlap on one device
 * race (the host part is serialised, device work on different streams is
 * not).  The array keeps the last call's contents; the call clears what must
 * start at zero. */
#define SNC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int snc_resultant_y_noalloc(snc_ctx* ctx, const snc_bipoly* f, const snc_bipoly* g, void* stream,
                            snc_upoly* out);

/* Resultant and square-free gcd in one pass: the projection step of the
 * curve analysis (Section 2.1) needs R = res_y(f, g) and gcd(R, R') (R / gcd
 * is the square-free part).  One run of the prepared pipeline computes both:
 * the modular Euclid of gcd(R, R') runs on R mod p for the resultant's own
 * primes right after the interpolation, beside the Chinese remaindering
 * (a second stream), and a prime not
 * dividing lc(R) with a constant gcd mod p proves gcd(R, R') = gcd(cont R,
 * cont R') = cont R; otherwise the full modular gcd of R follows (as
 * snc_gcd_z_deriv).  The Euclid's descriptors and outputs live in the
 * prepared workspace (its size from snc_resultant_y_batch_plan includes them).
 * R: the n resultants (conventions of snc_prepared_run).  G: the n gcds
 * (conventions of snc_gcd_z), sized by snc_prepared_sqfree_plan (gcd_each:
 * per pair, or NULL), which also sizes d_gws, a second device workspace
 * (caller-owned, not retained) for the full gcd when it is needed. */
int snc_prepared_sqfree_plan(const snc_prepared* prep, snc_plan* gcd_each, snc_plan* gcd_total);
int snc_prepared_run_sqfree(snc_prepared* prep, void* d_gws, size_t gws_bytes, void* stream, snc_upoly* R,
                            snc_upoly* G);

/* The Euclid of the square-free check (Section 2.1, gcd(R, R') mod p for
 * each of the resultant's primes; Section 4, "Symbolic Speedups").
 * snc_set_gcd_variant: 0 = automatic (one wavefront per (pair, prime), the
 * faster of the two on gfx950), 1 = one wavefront, 2 = the blocked Euclid
 * where the resultant degree needs 6, 9, 12 or 16 register slots per lane
 * (a workgroup of eight wavefronts per (pair, prime): a leading wavefront
 * decides blocks of up to 31 steps from the top 64 coefficients, another
 * accumulates each block's 2x2 polynomial matrix, the others apply the
 * previous block's matrix to the full remainders).  The variants give
 * identical degrees.  snc_prepared_sqfree_degrees: after snc_prepared_run_sqfree, for
 * pair `pair` and the first min(k, cap) of its k primes (the resultant's,
 * snc_prime(0), snc_prime(1), ...): d[q] = deg (R mod p_q) and e[q] = deg
 * gcd(R mod p_q, R' mod p_q) (-1 when R = 0 mod p_q; -2 marks a result to be
 * ignored).  Returns k (0 for a pair without a Euclid: trivial, or deg R < 1),
 * SNC_EINVAL before the first projection step or for a bad argument. */
int snc_set_gcd_variant(snc_ctx* ctx, int variant);
int snc_prepared_sqfree_degrees(const snc_prepared* prep, int pair, int32_t* d, int32_t* e, int cap);

/* Square-free factorisation (Section 2.1: R's square-free part and the
 * multiplicities of its real roots come from Yun's algorithm on R):
 *   a = content * prod_i f_i^{m_i},
 * content = cont(a) with the sign of lc(a) (0 for a = 0), the f_i primitive
 * with positive leading coefficients, square-free and pairwise coprime,
 * m_1 < m_2 < ....  Each step of Yun's algorithm is one modular gcd
 * (snc_gcd_z) whose lifted cofactors give the exact quotients.
 * plan: deg_bound = deg a, out_nlimbs = limbs per output coefficient (a bound
 * for every factor and the content), workspace_bytes = device workspace for
 * the steps.  run: content receives nlimbs limbs; the factors' coefficients
 * (ascending) go to limbs, concatenated, factor i taking degs[i] + 1
 * coefficients of nlimbs limbs each; mults[i] is its multiplicity;
 * *nfactors their number.  cap_coefs = 2 deg a + 1 and max_factors = deg a
 * always suffice; smaller capacities give SNC_ERANGE with *nfactors set.
 * SNC_ENOMEM if a step needs more workspace (the message says how much). */
int snc_sqfree_plan(const snc_upoly* a, snc_plan* out);
int snc_sqfree(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, void* stream, int32_t nlimbs,
               uint32_t* content, uint32_t* limbs, int32_t cap_coefs, int32_t* degs, int32_t* mults,
               int32_t max_factors, int32_t* nfactors);

/* Content of f in y (opening of Section 2.1: a curve's rows share a content h
 * whose real roots are vertical lines; the analysis divides it out first):
 *   h = gcd(f_0, f_1, ..., f_dy) in Z[x], f = sum_i f_i(x) y^i,
 * normalised to a positive leading coefficient (integer content included);
 * the zero polynomial (deg -1) for f = 0, the row itself (sign normalised)
 * when f has one non-zero row.  The rows are paired and their gcds taken in
 * one batched modular gcd (snc_gcd_z_batch) per level of a binary tree.
 * plan: deg_bound = the least row degree, out_nlimbs bounds h (Mignotte),
 *   workspace_bytes = the first level's batch.
 * run: out as for snc_gcd_z; SNC_ENOMEM if a later level needs more
 *   workspace (the message says how much). */
int snc_content_y_plan(const snc_bipoly* f, snc_plan* out);
int snc_content_y(snc_ctx* ctx, const snc_bipoly* f, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out);

/* Contents in y of n curves at once (opening of Section 2.1, for every curve
 * of a set): one binary tree over all curves, each level pairing the rows
 * of every curve and taking all pairs' gcds in one batched modular gcd
 * submission.  out[i] as snc_content_y of curve i.  plan: out_each[i] bounds
 * curve i's content (deg_bound, out_nlimbs), out_total the largest of them
 * and workspace_bytes the first level's batch; a later level that needs
 * more gives SNC_ENOMEM with the size in the message. */
int snc_content_y_batch_plan(int32_t n, const snc_bipoly* f, snc_plan* out_each, snc_plan* out_total);
int snc_content_y_batch(snc_ctx* ctx, int32_t n, const snc_bipoly* f, void* d_ws, size_t ws_bytes, void* stream,
                        snc_upoly* out);

/* Arrangement batch (Section 3: the projection phase of an arrangement of
 * curves C_1..C_n needs R_C = res(f, f_y, y) of every curve, after its
 * content in y is removed, and R_CD = res(f, g, y) of every pair).
 * prepare: the contents h_i = cont_y(f_i) of all curves in one tree of
 *   batched gcds (d_ws: workspace of snc_content_y_batch_plan), then on the
 *   host the primitive parts p_i = f_i / h_i (exact division of the rows)
 *   and their y-derivatives; the handle keeps them (inputs not retained).
 * plan: content_each[i] = the exact size of h_i (n entries, or NULL);
 *   res_each / res_total as snc_resultant_y_batch_plan for the n + n(n-1)/2
 *   resultants, in this order: res_y(p_i, dp_i/dy) for i = 0..n-1, then
 *   res_y(p_i, p_j) for i < j in lexicographic order.
 * run: contents (n) and resultants (n + n(n-1)/2) as snc_upoly outputs; all
 *   resultants run as one prepared batch (one graph replay), prepared on the
 *   first run with d_ws (which must stay valid until the handle is
 *   destroyed or a run with another workspace) and replayed afterwards. */
typedef struct snc_arrangement snc_arrangement;
int snc_arrangement_prepare(snc_ctx* ctx, int32_t n, const snc_bipoly* curves, void* d_ws, size_t ws_bytes,
                            void* stream, snc_arrangement** out);
int snc_arrangement_plan(const snc_arrangement* arr, snc_plan* content_each, snc_plan* res_each,
                         snc_plan* res_total);
int snc_arrangement_run(snc_arrangement* arr, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* contents,
                        snc_upoly* resultants);
int snc_arrangement_destroy(snc_arrangement* arr);

/* FastLift's second resultant (Section 2.1, "Lifting Phase", the bound
 * m*_alpha): with h = gcd(f_x, f_y) in Z[x, y], Q = res_y(f_x / h, f_y / h).
 * mult(Q, alpha) bounds the number of distinct complex roots of f(alpha, y):
 * m*_alpha = deg_y f - mult(R, alpha) + mult(Q, alpha).  A prime p and a
 * point x0 where gcd(f_x(x0, y), f_y(x0, y)) mod p is constant (and neither
 * leading coefficient in y vanishes) certify that deg_y h = 0; then h is the
 * gcd of all rows of f_x and f_y in Z[x] (snc_content_y's tree of batched
 * gcds).  Otherwise h depends on y and comes from a bivariate modular gcd
 * (Brown's dense method): contents in y and gamma = gcd of the leading
 * coefficients in Z[x] by the batched gcd, then on the device, per (prime,
 * point), gamma(x0) times the monic gcd in y of f_x(x0, y), f_y(x0, y)
 * mod p, interpolated in x and combined over primes by the resultant's own
 * kernels; the primitive part of the result, times the gcd of the
 * contents, is h once it divides f_x and f_y exactly (otherwise more primes
 * or other points are taken).  h is normalised to a positive leading
 * coefficient (in y, then in x), f_x and f_y are divided by h exactly on
 * the host, and Q comes from snc_resultant_y.
 * plan: the plan of res_y(f_x, f_y), an upper bound when h = +-1, with the
 *   workspace of the bivariate gcd's device pass; a non-trivial h may need
 *   more (SNC_ENOMEM / SNC_ERANGE with sizes, as for snc_resultant_y).
 * run: out as for snc_resultant_y. */
int snc_fastlift_q_plan(const snc_bipoly* f, snc_plan* out);
int snc_fastlift_q(snc_ctx* ctx, const snc_bipoly* f, void* d_ws, size_t ws_bytes, void* stream, snc_upoly* out);

/* ---- gcd in Z[x] ---------------------------------------------------------
 * Modular (small primes) gcd: contents on the host, monic gcd and cofactors
 * mod each prime on the device, primes of minimal gcd degree kept, CRT, and
 * an exact certificate (norm bound on the lifted product) before the result
 * is accepted; unlucky primes are replaced by more primes. */
/* gcd(a, b) of a, b in Z[x] (see snc_upoly), normalised to a positive
 * leading coefficient; the zero polynomial (deg -1) when a = b = 0.
 * plan: deg_bound and out_nlimbs bound the result, workspace_bytes sizes
 *   d_ws (0: the result needs no device work).
 * d_ws: device workspace of ws_bytes, caller-owned, not retained; SNC_ENOMEM
 *   if smaller than the plan asks.  out: caller-allocated; on SNC_ERANGE
 *   out->deg and out->nlimbs hold the sizes needed and nothing is written.
 * stream: HIP stream for the device work; the call returns when the result
 *   is in out (host memory). */
int snc_gcd_z_plan(const snc_upoly* a, const snc_upoly* b, snc_plan* out);
int snc_gcd_z(snc_ctx* ctx, const snc_upoly* a, const snc_upoly* b, void* d_ws, size_t ws_bytes,
              void* stream, snc_upoly* out);

/* n gcds in one submission.  The problems advance together in rounds: per
 * round one upload, one reduction launch, one Euclid launch per register
 * class and one download serve every unfinished problem; those with enough
 * primes of minimal gcd degree are then lifted and certified, the others
 * draw more primes.  a, b, out and out_each are arrays of n; out[i] receives
 * gcd(a[i], b[i]) with the conventions of snc_gcd_z.  On SNC_ERANGE each
 * entry that is too small holds the sizes it needs and no entry is valid.
 * out_total->workspace_bytes sizes d_ws for the whole batch (out_each: the
 * per-problem plans, or NULL).  Any invalid input fails the whole call. */
int snc_gcd_z_batch_plan(int32_t n, const snc_upoly* a, const snc_upoly* b, snc_plan* out_each,
                         snc_plan* out_total);
int snc_gcd_z_batch(snc_ctx* ctx, int32_t n, const snc_upoly* a, const snc_upoly* b, void* d_ws,
                    size_t ws_bytes, void* stream, snc_upoly* out);

/* gcd(a, a') with a' the formal derivative of a, formed inside the library:
 * the square-free part of the resultant R in the projection phase
 * (Section 2.1) is R / gcd(R, R').  Same conventions as snc_gcd_z. */
int snc_gcd_z_deriv_plan(const snc_upoly* a, snc_plan* out);
int snc_gcd_z_deriv(snc_ctx* ctx, const snc_upoly* a, void* d_ws, size_t ws_bytes, void* stream,
                    snc_upoly* out);

/* ---- serving --------------------------------------------------------------
 * A request loop with continuous batching.  The server owns the device pool
 * (d_pool, pool_bytes; caller-allocated, valid until snc_server_destroy) and
 * nstreams worker threads, each with its own context and HIP stream.
 * Submitting copies and plans the inputs (their device footprint is the
 * plan's workspace size; a request larger than the pool is refused with
 * SNC_ENOMEM).  A free worker admits the waiting resultant requests that fit
 * into the free pool bytes and the max_slots limit and runs them as one
 * batch, or runs one gcd; work on different streams overlaps on the device.
 * snc_poll returns SNC_EAGAIN until the request is finished, then writes the
 * result like the synchronous calls and releases the request (SNC_ERANGE
 * keeps it).  snc_request_times gives its submit and finish times (steady
 * clock, seconds), also after it was polled.  snc_server_wait blocks until
 * at least `completed` requests have finished since creation (SNC_EAGAIN on
 * timeout).  All server functions are thread-safe. */
int snc_server_create(snc_ctx* ctx, void* d_pool, size_t pool_bytes, int32_t max_slots, int32_t nstreams,
                      snc_server** out);
int snc_submit_resultant_y(snc_server* srv, const snc_bipoly* f, const snc_bipoly* g, uint64_t* ticket);
int snc_submit_gcd_z(snc_server* srv, const snc_upoly* a, const snc_upoly* b, uint64_t* ticket);
int snc_poll(snc_server* srv, uint64_t ticket, snc_upoly* out);
int snc_request_times(snc_server* srv, uint64_t ticket, double* submit_s, double* done_s);
int snc_server_wait(snc_server* srv, int64_t completed, double timeout_s);
int snc_server_destroy(snc_server* srv);

/* ---- host-side helpers (no device work) --------------------------------- */
/* i-th prime of the modulus table (descending below 2^30), 0 if out of range. */
uint32_t snc_prime(int32_t i);

#ifdef __cplusplus
}
#endif

#endif /* SNC_H */
