/*
 * libsfft -- encrypted fixed-point FFT over GSW13 (q = 2^k) on gfx950.
 *
 * The calls follow the paper's client/server workflow (Shortell and
 * Shokoufandeh, "Secure Fast Fourier Transform using Fully Homomorphic
 * Encryption", section "Introduction" and its cloud-computing figure): the
 * client generates keys (step 1) and encrypts its signal bit by bit (step 2);
 * the server evaluates the FFT on the ciphertexts (step 4); the client
 * decrypts (step 6).  Steps 3 and 5 (transport) are the caller's business.
 *
 * Scheme (section "Notation and Background"): Gentry-Sahai-Waters 2013 over
 * LWE, q = 2^k, ell = k bits per element, ciphertext dimension
 * Nct = (n+1)k, m = Nct, errors in {-1,0,1}.  A ciphertext is stored packed:
 * Nct rows, each n+1 elements of k/32 little-endian uint32 limbs
 * (Nct*Nct/8 bytes); its bits are the flattened binary ciphertext.
 * THE SIZES USED HERE ARE NOT SECURE: k is sized for correctness (noise)
 * only and the LWE dimension is tiny.
 *
 * A second family of calls (sfft_ring_*) works with the ring instantiation
 * of the same scheme over Z_p[X]/(X^d+1), p = 2^62 - 2^16 + 1: gates, blind
 * rotation, refresh of LWE ciphertexts mod p, bootstrapped gates, and FFT
 * plans evaluated on bootstrapped gates, whose parameters do not depend on
 * the circuit's depth (the same warning about security applies).
 *
 * Conventions for every call:
 *  - return value 0 (SFFT_OK) or a negative status; nothing is thrown across
 *    the ABI; sfft_last_error() gives a thread-local message for the last
 *    failure;
 *  - the caller owns every buffer it passes (host or device); the library
 *    never frees or retains caller memory; plans own only their own
 *    immutable tables;
 *  - `hip_stream` is a hipStream_t (NULL = the null stream); device calls are
 *    asynchronous on it unless stated; device faults surface as SFFT_EDEVICE
 *    from a later call or synchronisation.
 */
#ifndef SFFT_H
#define SFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SFFT_OK 0
#define SFFT_EINVAL (-1)        /* bad argument or shape */
#define SFFT_ENOMEM (-2)        /* host or device allocation failed */
#define SFFT_EDEVICE (-3)       /* HIP runtime error */
#define SFFT_ENOISE (-4)        /* k too small for the circuit's noise bound */
#define SFFT_EUNSUPPORTED (-6)  /* valid but not implemented (e.g. eta != 1) */

/* Scheme parameters: q = 2^k (k a positive multiple of 32), LWE dimension
 * n_lwe >= 1, m = (n_lwe+1)*k samples, eta = 1 (errors in {-1,0,1}). */
typedef struct {
    int32_t n_lwe, k, m, eta;
} sfft_params;

/* Transform shape: dims 1 (len points) or 2 (len x len image, rows then
 * columns); len a power of two in [2, 4096]; F-bit two's-complement words
 * with f fractional bits (1 <= F <= 32, 0 <= f <= F); is_complex 0 for real
 * input (imaginary parts are plaintext zero and not encrypted).  nand_only 1
 * builds the paper's literal circuit, every gate a NAND (Lemma "binary
 * gates"; full adders as two half adders and an OR, Lemma "full adder"),
 * instead of the arithmetic gate forms (0, the default). */
typedef struct {
    int32_t dims, len, F, f, is_complex;
    int32_t nand_only;
} sfft_shape;

typedef struct sfft_plan sfft_plan;

/* Statistics of a compiled plan. */
typedef struct {
    int64_t nodes;          /* gates of the canonical netlist incl. inputs and NOTs */
    int64_t gates;          /* AND + XOR + OR + XADD of the canonical netlist */
    int64_t products;       /* distinct ciphertext products of the canonical netlist */
    int64_t exec_products;  /* product items the plan executes (after sharing) */
    int64_t levels;         /* product depth (launches) */
    int64_t max_level_products;
    int64_t n_inputs, n_outputs;  /* ciphertexts */
    int64_t ws_cts;               /* workspace ciphertext slots */
    int64_t exec_steps;           /* steps of sfft_execute_steps: levels + 2 */
    int32_t k_required;           /* least multiple of 32 meeting the noise rule */
    char netlist_sha256[65];      /* hex SHA-256 of the canonical netlist */
    int32_t tiling;               /* product-kernel tiling the plan launches (sfft_tiling_describe) */
    int64_t prod_ct_reads;        /* ciphertexts the product items read: L, R and extra operands */
    int64_t prod_ct_writes;       /* ciphertexts the product items write (their outputs) */
    int64_t ws_bytes;             /* workspace bytes sfft_execute needs (= sfft_plan_workspace_bytes):
                                     ws_cts slots, then the matrix-core kernel's copies of one level's
                                     right operands */
    int32_t noise_bound_bits;     /* bit length of the worst-case output noise bound at this Nct
                                     (k must exceed it by 3: the noise rule) */
} sfft_plan_info;

const char* sfft_last_error(void);

/* Least k (multiple of 32) for which every output's worst-case noise of the
 * shape's canonical circuit stays below q/8 at n_lwe (Lemmas "encryption",
 * "decryption", "evaluation": decryption is correct while noise < q/4).
 * Fills out->{n_lwe, k, m = (n_lwe+1)k, eta = 1}. */
int sfft_size_params(const sfft_shape* shape, int32_t n_lwe, sfft_params* out);

/* Bytes of one ciphertext: Nct*Nct/8.  Negative status on bad params. */
int64_t sfft_ct_bytes(const sfft_params* params);

/* Key generation (workflow step 1).  pk_host: m x (n+1) elements, k/32 limbs
 * each (sfft_ct_bytes bytes) = A = [B t + e | B]; sk_host: (n+1) elements of
 * k/32 limbs = s = (1, -t).  Deterministic in seed (SplitMix64 domains 1-3). */
int sfft_keygen(const sfft_params* params, uint64_t seed, uint32_t* pk_host, uint32_t* sk_host);

/* Encryption (workflow step 2, Lemma "encryption"): each of n_values F-bit
 * words (fixed_host, low F bits used) becomes F ciphertexts, LSB first:
 * ciphertext i = value i/F, bit i%F; C' = mu G + R A with R drawn from
 * SplitMix64 domain 4 at ciphertext id first_ct_id + i.  pk_dev: the public
 * key in device memory; ct_dev: n_values*F ciphertexts (device). */
int sfft_encrypt(const sfft_params* params, const uint32_t* pk_dev, const int32_t* fixed_host, int64_t n_values,
                 int32_t F, uint64_t seed, uint64_t first_ct_id, uint32_t* ct_dev, void* hip_stream);

/* Compile the FFT circuit for a shape (Theorem 1 / Lemma "evaluation": bit
 * reversal, then log2 N butterfly stages of additions, subtractions and
 * constant multiplications), levelise it and upload its work tables.  Fails
 * with SFFT_ENOISE if params->k is below the circuit's requirement. */
int sfft_plan_create(const sfft_shape* shape, const sfft_params* params, sfft_plan** out);
int sfft_plan_info_get(const sfft_plan* plan, sfft_plan_info* info);
/* Host-only compilation of the same circuit: fills `info` without touching
 * any device (no allocation, no HIP call).  Same errors as plan creation. */
int sfft_analyze(const sfft_shape* shape, const sfft_params* params, sfft_plan_info* info);
/* The same circuit with its workspace bounded by ws_limit_bytes (0: no
 * bound, the plan of sfft_plan_create).  Levels are then formed by list
 * scheduling instead of as soon as possible: products in order of first
 * appearance in the netlist (the first rows' and stages' butterflies first),
 * a level taking ready products while the workspace ciphertexts live
 * through it fit the bound.  More levels of fewer products; the same
 * ciphertexts.  sfft_plan_info.ws_bytes is the bounded workspace;
 * SFFT_ENOMEM if the circuit cannot run within the bound. */
int sfft_plan_create_bounded(const sfft_shape* shape, const sfft_params* params, int64_t ws_limit_bytes,
                             sfft_plan** out);
int sfft_analyze_bounded(const sfft_shape* shape, const sfft_params* params, int64_t ws_limit_bytes,
                         sfft_plan_info* info);
/* Device workspace the caller must pass to sfft_execute. */
int sfft_plan_workspace_bytes(const sfft_plan* plan, int64_t* bytes);
/* Waits for all device work (work enqueued with the plan reads its tables),
 * then frees the plan. */
void sfft_plan_destroy(sfft_plan* plan);

/* Encrypted FFT (workflow step 4).  ct_in_dev: the shape's input ciphertexts,
 * id (v*C + comp)*F + bit (v = point, row-major for images; C = 2 complex or
 * 1 real; comp 0 = Re, 1 = Im); ct_out_dev: len (1D) or len*len (2D) complex
 * outputs in natural order, id (v*2 + comp)*F + bit.  ws_dev: at least
 * sfft_plan_workspace_bytes.  Enqueues only. */
int sfft_execute(const sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                 int64_t ws_bytes, void* hip_stream);

/* The same work split into exec_steps ordered steps: step 0 prepares inputs
 * (linear gates on inputs), step L in [1, levels] runs product level L and
 * the linear gates that follow it, the last step writes outputs that are
 * constants, inputs or repeated.  Running every step in order equals
 * sfft_execute; between steps the caller may enqueue other work (other
 * requests' steps, timing events) on the same or other streams. */
int sfft_execute_steps(const sfft_plan* plan, int32_t first, int32_t count, const uint32_t* ct_in_dev,
                       uint32_t* ct_out_dev, void* ws_dev, int64_t ws_bytes, void* hip_stream);
/* sfft_execute through a HIP graph: the first call (or one with other
 * buffers than the last) captures the plan's launch sequence on hip_stream
 * (which must not be the null stream) and instantiates it; later calls with
 * the same buffers replay it with one graph launch.  One captured graph per
 * plan; the graph holds no memset nodes.  Same results as sfft_execute. */
int sfft_execute_graph(sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                       int64_t ws_bytes, void* hip_stream);
/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * as sfft_execute with the workspace in a fixed array of the library's own
 * device memory, SFFT_NOALLOC_WS_BYTES (64 MiB) on each GPU it runs on, held
 * until the process ends.  It allocates and frees nothing.  SFFT_ENOMEM if
 * the plan's workspace (sfft_plan_workspace_bytes) is larger.  Every call on
 * one GPU uses the same array, so calls that overlap on one GPU race:
 * enqueue them on one stream, or let one finish before the next starts.
 * Enqueues only. */
#define SFFT_NOALLOC_WS_BYTES (64ll << 20)
int sfft_execute_noalloc(const sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* hip_stream);
/* sfft_execute in one persistent launch, for small plans whose levels are
 * too small to fill the GPU (a kernel boundary per level then costs about as
 * much as the level): a cooperative launch of the 256-thread matrix-core
 * kernel that transposes R in the workgroup (where its LDS holds every chunk
 * of R: Nct up to 512 or 1024 by fragments per wave), else of the 512-thread
 * one with in-kernel transposition; as many workgroups as are resident at
 * once (at most what the widest level uses) loop over every level's
 * product tiles and linear items with a grid-wide barrier between levels
 * (agent-scope release and acquire around a counter).  The barrier's waits
 * are bounded (about 0.1 s): one that runs out sets a flag
 * (sfft_plan_persistent_timeouts) instead of hanging.  The first call
 * uploads the plan's level tables and allocates its barrier words.
 * SFFT_EUNSUPPORTED for rows of more than 8 fragments (4 W > 256 bytes).
 * Same ciphertexts as sfft_execute.  Executions on one plan must not
 * overlap (they share the barrier words). */
int sfft_execute_persistent(sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                            int64_t ws_bytes, void* hip_stream);
/* Waits for the device; *flag = 1 if a barrier wait of a persistent
 * execution on this plan ran out since its last launch began, else 0. */
int sfft_plan_persistent_timeouts(sfft_plan* plan, int32_t* flag);
/* Measurement aid.  With enable != 0, every later sfft_execute_steps (and
 * sfft_execute) call on this plan records a pair of HIP events on its stream
 * around each level's product kernel alone (after the right operands'
 * transposition, before the level's linear gates); enable = 0 stops it.  Not
 * for graph capture, and not thread-safe with other calls on the plan. */
int sfft_plan_time_products(sfft_plan* plan, int32_t enable);
/* Waits for the recorded pairs, returns the sum of their elapsed times (ms)
 * and their number, and releases them. */
int sfft_plan_product_time(sfft_plan* plan, double* total_ms, int64_t* launches);
/* Fixed batches: a set of requests known in advance, merged level by level
 * as the request loop merges them (global step s advances every request
 * that has a step s; the products of all requests whose kernel tiling
 * matches run in one launch, one segment per request with its own
 * geometry; then the linear passes), but compiled once: every step's
 * segment lists are uploaded at creation into one device table, so an
 * execution is the launch sequence alone (section "FFT in FHE": the
 * butterflies of a stage, and independent requests, run side by side).
 * Each request's ciphertexts equal those of its plan run alone.  plans,
 * ct_in_dev, ct_out_dev: n entries (request r runs plans[r] from ct_in_dev[r]
 * into ct_out_dev[r], layouts of sfft_execute); the plans must outlive the
 * batch.  ws_dev: at least sfft_batch_workspace_bytes, each request's
 * workspace in its own 256-byte-aligned part.  The buffers are fixed for the
 * batch's life. */
typedef struct sfft_batch sfft_batch;
int sfft_batch_workspace_bytes(const sfft_plan* const* plans, int32_t n, int64_t* bytes);
int sfft_batch_create(const sfft_plan* const* plans, const uint32_t* const* ct_in_dev, uint32_t* const* ct_out_dev,
                      int32_t n, void* ws_dev, int64_t ws_bytes, sfft_batch** out);
/* Global steps and launches of one execution. */
int sfft_batch_info(const sfft_batch* batch, int64_t* steps, int64_t* launches);
/* Enqueues the launch sequence on hip_stream. */
int sfft_batch_execute(const sfft_batch* batch, void* hip_stream);
/* The same through a HIP graph: the first call captures the sequence on
 * hip_stream (not the null stream) and instantiates it; every call launches
 * it with one graph launch.  The graph holds no memset nodes. */
int sfft_batch_execute_graph(sfft_batch* batch, void* hip_stream);
/* Waits for the device, then frees the batch's table and graph. */
void sfft_batch_destroy(sfft_batch* batch);
/* Product items per step (counts has exec_steps entries). */
int sfft_plan_step_products(const sfft_plan* plan, int64_t* counts, int32_t n);

/* Decryption (workflow step 6, Lemma "decryption"): n_values words of F
 * ciphertexts each (LSB first) -> signed values sign-extended from F bits.
 * ct: host or device (ct_on_device = 1; reads row k-1 of each ciphertext and
 * synchronises the null stream). */
int sfft_decrypt(const sfft_params* params, const uint32_t* sk_host, const uint32_t* ct, int64_t n_values,
                 int32_t F, int ct_on_device, int32_t* fixed_out);
/* sfft_decrypt of device ciphertexts whose rows k-1 are read on hip_stream
 * alone (an asynchronous copy, then a wait for that stream only): work on
 * other streams keeps running.  The caller makes sure the ciphertexts are
 * complete (for example a request of the request loop that has finished,
 * sfft_server_poll). */
int sfft_decrypt_stream(const sfft_params* params, const uint32_t* sk_host, const uint32_t* ct_dev, int64_t n_values,
                        int32_t F, void* hip_stream, int32_t* fixed_out);
/* Measured noise (Lemma "decryption": C' s = mu G s + e, row r of G s being
 * 2^t s_b for r = b k + t): for each of n_ct device ciphertexts whose bits
 * are mu_bits, e_r = <C'_r, s> - mu 2^t s_b mod q, centred; *max_bits is the
 * bit length of the largest |e_r| over every row of every ciphertext (0 for
 * none).  Reads whole ciphertexts (Nct^2/8 bytes each) on hip_stream and
 * waits for that stream; the caller makes sure they are complete.  Host
 * arithmetic. */
int sfft_noise_bits(const sfft_params* params, const uint32_t* sk_host, const uint32_t* ct_dev, int64_t n_ct,
                    const int32_t* mu_bits, void* hip_stream, int32_t* max_bits);
/* Decryption of n_ct single bits. */
int sfft_decrypt_bits(const sfft_params* params, const uint32_t* sk_host, const uint32_t* ct, int64_t n_ct,
                      int ct_on_device, int32_t* bits_out);

/* Single gates on device ciphertexts (section "Notation and Background":
 * addition, multiplication and NAND of ciphertexts; Lemma "binary gates"):
 * gate = 3 NOT (y ignored), 4 AND, 5 XOR, 6 OR, 7 XADD (addition; the result
 * encrypts x+y, a bit only if x,y are never both 1), 8 NAND, 9 PRODUCT
 * (= AND).  x, y, out: one ciphertext each, device; out must not alias.
 * Allocates nothing and holds no shared state, so calls on different streams
 * may overlap. */
int sfft_gate(const sfft_params* params, int32_t gate, const uint32_t* x_dev, const uint32_t* y_dev,
              uint32_t* out_dev, void* hip_stream);

/* ---- product-kernel tilings and the autotuner ---------------------------
 * The gate product (section "Time/Space Complexities": a matrix-matrix
 * product per gate) has two kernels, each in several tilings: a table-lookup
 * kernel on the integer VALU (threads per workgroup, lanes per output row,
 * digit slots per lane, rows per lane, lookup pipeline depth, 4-bit groups
 * per chunk of R) and a matrix-core kernel that multiplies the bits of L by
 * the bytes of R with int8 MFMA (threads, row groups, column groups, 32-byte
 * column fragments per wave).  Plans use, per ciphertext geometry (k,
 * n_lwe), the tiling recorded for it (by sfft_tune or sfft_set_tiling,
 * process-wide), else the matrix-core default for the row width, else a
 * lookup default by digits per row.  Plans keep the tiling they were created
 * with.  Encryption always runs on the lookup kernel. */
int sfft_tiling_count(void);
/* fields[7]: fields[6] = 0 for a lookup tiling, then fields[0..5] = threads,
 * lanes per row, digit slots per lane, rows per lane, pipeline depth, groups
 * per chunk; fields[6] = 1 for a matrix-core tiling, then fields[0..4] =
 * threads, row groups, column groups, fragments per wave, and how the right
 * operands reach the kernel: 0 each workgroup transposes its chunks itself
 * (512-thread layout), 1 a pass before each launch transposes them into the
 * workspace in 128-row chunks, 2 the same in 64-row chunks (256-thread
 * kernel), 3 the 256-thread kernel's workgroup transposes all its chunks into
 * LDS itself (small products); fields[5] = 0.
 * SFFT_EINVAL for an unknown tiling. */
int sfft_tiling_describe(int32_t tiling, int32_t* fields);
/* Record a tiling for params' geometry (-1: back to the default).
 * SFFT_EINVAL if the tiling cannot serve the geometry. */
int sfft_set_tiling(const sfft_params* params, int32_t tiling);
/* Time every tiling that can serve params' geometry on a synthetic level of
 * products (random operands, two outputs each; reps timed launches after a
 * warm-up, on hip_stream), record the fastest and return it in
 * *best_tiling.  rates (optional, sfft_tiling_count() entries) receives
 * bit-MAC/s per tiling, 0 where a tiling cannot serve.  Allocates and frees
 * its own device buffers (a few GB at most); synchronous. */
int sfft_tune(const sfft_params* params, int32_t reps, int32_t* best_tiling, double* rates, void* hip_stream);
/* Tune on a plan's own work: run the plan's steps up to its widest product
 * level (ct_in_dev, ct_out_dev and the workspace as for sfft_execute), time
 * that level under every tiling that can serve the plan, switch the plan to
 * the fastest and record it for its geometry.  Re-running a level rewrites
 * the same outputs, so the buffers hold a valid partial run afterwards;
 * sfft_execute from the start gives the usual result.  Synchronous. */
int sfft_plan_tune(sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                   int64_t ws_bytes, int32_t reps, int32_t* best_tiling, double* rates, void* hip_stream);

/* ---- continuous batching / serving -------------------------------------
 * A server runs many encrypted FFTs of different shapes and parameter sets
 * at once.  Requests are admitted in arrival order when their plan's
 * workspace fits the device memory budget (and fewer than max_active run);
 * each global step advances every admitted request by one of its plan's
 * steps, with the products of all requests that share a kernel tiling (and
 * LDS occupancy) in one launch, whatever their k and n.  Each request's ciphertexts are bit-identical to running
 * its plan alone.  Requests are independent FFTs (the paper's workflow,
 * section "Introduction", repeated per client signal). */
#define SFFT_SERVER_DRYRUN 1  /* no device work: admission/scheduling only, modelled time */
#define SFFT_SERVER_SERIAL 2  /* a step's launches of different tilings in turn on the caller's stream
                                 (by default they overlap on the server's own streams) */

typedef struct {
    int64_t mem_budget_bytes;  /* device memory for request workspaces (allocated at create) */
    int32_t max_active;        /* requests in flight at once; 0 = no limit */
    int32_t flags;             /* SFFT_SERVER_DRYRUN, SFFT_SERVER_SERIAL */
    double dry_bitmac_per_s;   /* modelled product rate in dry-run mode (0 = 1e15) */
    /* 0: every step advances every admitted request (lockstep).  > 0: a step
     * advances admitted requests in order of least remaining work: the first
     * always, others while the step's product workgroups are below
     * fill_blocks, skipping any whose level alone exceeds fill_blocks.  The
     * others wait, so small requests are not held to the pace of a large
     * one's levels.  Admission then also lets a later request whose
     * workspace fits pass one that does not yet. */
    int64_t fill_blocks;
} sfft_server_cfg;

typedef struct {
    int64_t submitted, admitted, completed, queued, active;
    int64_t steps, launches, products, gates, fft_points;
    int64_t max_active, peak_ws_bytes;
    double clock_s; /* current time: host seconds, or modelled seconds in dry-run */
} sfft_server_stats;

typedef struct sfft_server sfft_server;

int sfft_server_create(const sfft_server_cfg* cfg, sfft_server** out);
/* Queue a request: the shape's input ciphertexts (layout of sfft_execute) in
 * ct_in_dev, outputs written to ct_out_dev; both caller-owned and untouched
 * by the caller until the request completes.  Compiles (or reuses) the plan
 * on the host.  SFFT_ENOMEM if the plan's workspace exceeds the budget. */
int sfft_server_submit(sfft_server* srv, const sfft_shape* shape, const sfft_params* params,
                       const uint32_t* ct_in_dev, uint32_t* ct_out_dev, uint64_t* ticket);
/* The same with a plan the caller already compiled (sfft_plan_create): no
 * host compilation on submit.  The plan is shared, not copied, and must
 * outlive the request. */
int sfft_server_submit_plan(sfft_server* srv, const struct sfft_plan* plan, const uint32_t* ct_in_dev,
                            uint32_t* ct_out_dev, uint64_t* ticket);
/* Admit what fits and enqueue one global step on hip_stream (launches of
 * different tilings overlap on the server's own streams, joined back on
 * hip_stream), without waiting for the device: the host runs up to four
 * steps ahead.  A request completes when the device has finished its last
 * step; its workspace then returns to the budget.  *pending = requests
 * still queued, running or finishing.  A request left out by the fill
 * policy for 8 steps in a row runs in the next one. */
int sfft_server_step(sfft_server* srv, void* hip_stream, int32_t* pending);
/* done = 1 once the request's outputs are complete; latency = completion
 * minus submission (seconds; modelled in dry-run). */
int sfft_server_poll(sfft_server* srv, uint64_t ticket, int32_t* done, double* latency_s);
/* Step until every submitted request is complete. */
int sfft_server_drain(sfft_server* srv, void* hip_stream);
int sfft_server_stats_get(const sfft_server* srv, sfft_server_stats* out);
/* Waits for all device work, then frees the server and its memory budget. */
void sfft_server_destroy(sfft_server* srv);

/* ---- ring-GSW gates ------------------------------------------------------
 * GSW13's ring instantiation of the scheme the paper evaluates its circuits
 * with (section "Notation and Background"; gates as in Lemma "binary gates"):
 * matrix entries are polynomials of R_p = Z_p[X]/(X^d + 1) with
 * p = SFFT_RING_P = 2^62 - 2^16 + 1 (prime, 2^16 | p - 1) and d a power of
 * two in [1, 2048].  With ell = SFFT_RING_ELL = 62 and v = (1, -s):
 *   ciphertext  C = m*G + Z, 2*ell rows x 2 columns of polynomials,
 *               G = I_2 (x) (1, 2, ..., 2^(ell-1))^T, row r of Z is
 *               (a_r*s + e_r, a_r), so C*v = m*G*v + e
 *   product     P = G^-1(L)*R, G^-1 = bit decomposition of every coefficient
 *   gates       AND = P, XOR = L + R - 2P, OR = L + R - P, NAND = G - P,
 *               NOT = G - L, XADD = L + R (codes as for sfft_gate)
 *   decryption  coefficient 0 of row ell-1 of C*v: |centred value| > p/4
 *               reads 1
 * Layout: (row, column, coefficient) uint64 residues in [0, p),
 * sfft_ring_ct_words(d) = 2*ell*2*d words per ciphertext, n ciphertexts back
 * to back.  Every call returns SFFT_EINVAL for a d outside the range, n < 0,
 * a null buffer or an unknown gate; n = 0 does nothing.  The first call for a
 * d on a device uploads that d's transform tables (the library's only
 * allocation here; kept until the process ends).  Launches are asynchronous
 * on hip_stream. */
#define SFFT_RING_P 0x3FFFFFFFFFFF0001ULL
#define SFFT_RING_ELL 62

/* Words per ring ciphertext, or SFFT_EINVAL. */
int64_t sfft_ring_ct_words(int32_t d);
/* Workspace of sfft_ring_gate for n product gates: the transformed right
 * operands, n * sfft_ring_ct_words(d) words. */
int sfft_ring_workspace_bytes(int32_t d, int64_t n, int64_t* bytes);
/* Encrypt n bits (bits_dev, one byte each, 0/1).  The random draws are
 * inputs, all on the device: s_dev the secret's d signed coefficients,
 * a_dev n*2*ell*d masks in [0, p), e_dev n*2*ell*d signed errors.  ct_dev
 * receives n ciphertexts. */
int sfft_ring_encrypt(int32_t d, const int64_t* s_dev, const uint64_t* a_dev, const int64_t* e_dev,
                      const uint8_t* bits_dev, int64_t n, uint64_t* ct_dev, void* hip_stream);
/* out[c] = gate(x[c], y[c]) for c < n, device buffers of n ciphertexts each;
 * out must not alias x or y (SFFT_EINVAL).  Product gates (4, 5, 6, 8, 9)
 * need a workspace of sfft_ring_workspace_bytes(d, n) bytes (SFFT_EINVAL if
 * smaller); NOT (3, y ignored) and XADD (7) need none. */
int sfft_ring_gate(int32_t d, int32_t gate, const uint64_t* x_dev, const uint64_t* y_dev, uint64_t* out_dev,
                   int64_t n, void* ws_dev, int64_t ws_bytes, void* hip_stream);
/* Decrypt n ciphertexts (host, or device with ct_on_device = 1: reads row
 * ell-1 of each, synchronously) under the secret's d signed coefficients. */
int sfft_ring_decrypt(int32_t d, const int64_t* s_host, const uint64_t* ct, int64_t n, int ct_on_device,
                      uint8_t* bits_out);

/* ---- blind rotation (the core of a refresh) --------------------------------
 * Refresh is only mentioned by the paper (section "Error Analysis"); this is
 * the step that FHEW/TFHE-style refresh is built on, written for the ring-GSW
 * ciphertexts above as the key.  A ring-LWE accumulator is a pair of
 * polynomials (b, a), 2*d words, encrypting b - a*s.  Blind rotation by a key
 * of n ring-GSW encryptions bk[i] of bits s_i and rotations r_i runs, for
 * i = 0..n-1, the CMux step
 *     acc <- acc + G^-1(X^r_i acc - acc) * bk[i]
 * so that acc ends encrypting X^(sum r_i s_i) times what it encrypted.  Each
 * step adds at most 2*ell*d times the key's error bound, whatever the
 * accumulator's own error: that is what makes refresh possible
 * (sfft_ring_bootstrap and sfft_ring_keyswitch complete it for LWE
 * ciphertexts mod p). */
/* Forward transforms of the key's rows into bkt_dev (n * sfft_ring_ct_words(d)
 * words, must not alias bk_dev); done once per key. */
int sfft_ring_bk_prepare(int32_t d, const uint64_t* bk_dev, int64_t n, uint64_t* bkt_dev, void* hip_stream);
/* Blind-rotate m accumulators in place (acc_dev: m * 2d words, device) by the
 * prepared key bkt_dev (n ciphertexts); rot_dev: m * n int32 rotations, row j
 * for accumulator j, taken mod 2d.  One launch; one workgroup per
 * accumulator runs its n steps in order. */
int sfft_ring_blind_rotate(int32_t d, const uint64_t* bkt_dev, int64_t n, const int32_t* rot_dev, uint64_t* acc_dev,
                           int64_t m, void* hip_stream);
/* Gate bootstrapping within the ring scheme (FHEW-style refresh without the
 * final key switch).  lwe_dev: m LWE ciphertexts mod p, n+1 words each
 * (a_0..a_{n-1}, b), under a binary secret of n bits s_i, encrypting mu in
 * {0,1} as b - <a,s> = mu*floor(p/2) + e with |e| < p/8 less the rounding of
 * the modulus switch.  bkt_dev: the prepared key of ring-GSW encryptions of
 * the s_i (sfft_ring_bk_prepare).  Steps: switch a, b to the modulus 2d
 * (floor((x*2d + floor(p/2))/p) mod 2d); accumulator
 * (X^(b~ + d/2) * Delta*(1 + X + ... + X^(d-1)), 0), Delta = floor(p/4);
 * blind rotation by -a~_i; coefficient 0 extracted.  out_dev: m LWE
 * ciphertexts of d+1 words (a'_0..a'_{d-1}, b') under the ring secret's
 * coefficients, a'_0 = a_0, a'_t = -a_{d-t}, b' = b_0 + Delta, whose phase is
 * mu*2*Delta plus the blind rotation's error only.  ws: at least
 * sfft_ring_bootstrap_workspace_bytes (accumulators and rotations). */
int sfft_ring_bootstrap_workspace_bytes(int32_t d, int64_t n, int64_t m, int64_t* bytes);
int sfft_ring_bootstrap(int32_t d, const uint64_t* bkt_dev, int64_t n, const uint64_t* lwe_dev, int64_t m,
                        uint64_t* out_dev, void* ws_dev, int64_t ws_bytes, void* hip_stream);
/* Key switching from the ring secret back to the LWE secret, which closes the
 * refresh loop: in_dev holds m LWE ciphertexts of d+1 words under the ring
 * secret's coefficients (sfft_ring_bootstrap's output), out_dev receives m of
 * n+1 words under the LWE secret of the key-switching key.  ksk_dev: d x 16 x
 * (n+1) words, entry [t][k] an LWE encryption (a_0..a_{n-1}, b) of
 * s_ring[t] * 16^k (caller-made, like the key).  out = (0, .., 0, b') -
 * sum_{t,k} digit_k(a'_t) * ksk[t][k], digit_k the base-16 digits.  The error
 * added is at most d*16*15 times the key's. */
int sfft_ring_keyswitch(int32_t d, int64_t n, const uint64_t* ksk_dev, const uint64_t* in_dev, int64_t m,
                        uint64_t* out_dev, void* hip_stream);
/* Bootstrapped binary gates (FHEW-style: every gate refreshes, so circuits
 * of any depth decrypt).  x_dev, y_dev: m LWE ciphertexts mod p of n+1 words
 * under the LWE secret, bits encoded as mu * 2 * floor(p/8) (error below
 * p/16).  gate: 4 AND, 5 XOR, 6 OR, 8 NAND.  Each output is
 *   keyswitch(bootstrap(cx*x + cy*y + (0, .., 0, k*floor(p/8))))
 * with (cx, cy, k) = (1, 1, -1) AND, (1, 1, 1) OR, (-1, -1, 5) NAND,
 * (2, 2, 0) XOR, and the bootstrap's accumulator value floor(p/8) (in place
 * of sfft_ring_bootstrap's floor(p/4)), so out_dev (m x (n+1) words) holds
 * the gate's bit in the same encoding under the same secret.  ws: at least
 * sfft_ring_gate_bootstrap_workspace_bytes.  NOT needs no bootstrap:
 * (0, .., 0, 2*floor(p/8)) - x. */
int sfft_ring_gate_bootstrap_workspace_bytes(int32_t d, int64_t n, int64_t m, int64_t* bytes);
int sfft_ring_gate_bootstrap(int32_t d, int32_t gate, const uint64_t* bkt_dev, int64_t n, const uint64_t* ksk_dev,
                             const uint64_t* x_dev, const uint64_t* y_dev, int64_t m, uint64_t* out_dev, void* ws_dev,
                             int64_t ws_bytes, void* hip_stream);
/* Encrypted FFT plans on bootstrapped gates: the shape's canonical netlist
 * (as for sfft_plan_create; shared nodes merged) evaluated gate by gate on
 * LWE ciphertexts mod p of n+1 words, every binary gate a
 * sfft_ring_gate_bootstrap gate, so the circuit's depth puts no bound on the
 * parameters.  Binary nodes are levelised (NOT is free and takes its
 * operand's level); one batched bootstrapped call per level, whatever the
 * mix of gate kinds (every row carries its gate code), then the level's NOTs.
 * Input ciphertext order is that of sfft_execute (value, component, bit LSB
 * first), bits encoded as mu * 2 * floor(p/8) under the LWE secret; outputs
 * likewise, always complex.  The workspace holds a slot of n+1 words per node
 * and one call's scratch. */
typedef struct sfft_ring_plan sfft_ring_plan;
typedef struct {
    int64_t nodes, gates;      /* netlist nodes; binary gates (= bootstraps per FFT) */
    int32_t levels, calls;     /* gate levels; batched gate calls per FFT */
    int64_t max_batch;         /* the largest call's gates */
    int64_t n_inputs, n_outputs;
    int64_t ws_bytes;
} sfft_ring_plan_info;
/* Host only: the plan's figures without building it on a device. */
int sfft_ring_plan_analyze(const sfft_shape* shape, int32_t d, int64_t n, sfft_ring_plan_info* info);
int sfft_ring_plan_create(const sfft_shape* shape, int32_t d, int64_t n, sfft_ring_plan** out);
/* bkt_dev: prepared key of the n LWE secret bits (sfft_ring_bk_prepare);
 * ksk_dev: key-switching key (sfft_ring_keyswitch).  Asynchronous on
 * hip_stream. */
int sfft_ring_fft_execute(const sfft_ring_plan* plan, const uint64_t* bkt_dev, const uint64_t* ksk_dev,
                          const uint64_t* in_dev, uint64_t* out_dev, void* ws_dev, int64_t ws_bytes, void* hip_stream);
void sfft_ring_plan_destroy(sfft_ring_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* SFFT_H */
