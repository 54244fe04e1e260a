/*
 * mmp.h -- exact modular matrix multiplication C = A B mod p on MI355X (gfx950).
 *
 * The method is the multiword floating-point product of Berthomieu, Graillat,
 * Lesnoff and Mary, "Multiword matrix multiplication over large finite fields
 * in floating-point arithmetic":
 *   - A and B are split into u and v words, A = sum_i alpha^i A_i and
 *     B = sum_j beta^j B_j with alpha = ceil(p^(1/u)), beta = ceil(p^(1/v))
 *     (Section 3.1, Alg. 4);
 *   - the uv word products A_i B_j are accumulated in binary64, reduced mod p
 *     with the fma-based reduction (Section 2.1, Alg. 1) after every k-block
 *     whose length respects the block-size bound (Section 2.2, Prop.
 *     blockProduct; Section 3.2, Prop. UVMW, eq. cAcB);
 *   - the products are recombined mod p (Section 3.2, eq. for AB as a sum
 *     over (i, j) of alpha^i beta^j A_i B_j), here by a Horner scheme with the
 *     modular product reduction (Section 2.1, Alg. 2).
 *
 * Conventions for every entry point below:
 *   - Matrices are row-major.  A is m x k with leading dimension lda >= k,
 *     B is k x n with ldb >= n, C is m x n with ldc >= n.
 *   - FP64 matrices hold integers in [0, p) (the representation of F_p used
 *     throughout the paper).  Results are bit-exact: C[i][j] is the unique
 *     integer in [0, p) congruent to sum_l A[i][l] B[l][j], stored as +0.0 ..
 *     p-1 in binary64.
 *   - Matrix pointers are DEVICE pointers (memory of the current HIP device).
 *     The caller owns A, B and C and keeps them alive until the call has
 *     completed in stream order.  C must not overlap A or B.
 *   - A stream argument is a hipStream_t passed as void*; NULL is the null
 *     stream.  Calls with a stream are asynchronous unless stated otherwise.
 *   - The modulus must satisfy 5 <= p < 2^52 (the paper assumes p >= 5 and
 *     Alg. 1 needs p < 2^(t-1) with t = 53).  Primality is not required: the
 *     recombination used here needs no modular inverse.
 *   - m, n or k may be 0; with k = 0 the result C is all zeros.
 *   - Errors are returned as negative mmp_status values; no entry point
 *     aborts or lets a C++ exception escape.
 */
#ifndef MMP_H
#define MMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MMP_OK = 0,
  MMP_EINVAL = -1,      /* null pointer, negative size, bad leading dimension,
                           p outside [5, 2^52), unsupported (u, v) or option */
  MMP_EBOUND = -2,      /* the requested (u, v) admits no block size >= 1 for
                           this p, or a forced k-block exceeds the bound */
  MMP_ERANGE = -3,      /* entry validation found an entry outside [0, p) or
                           a non-integral entry */
  MMP_ENOMEM = -4,      /* device or host allocation failed */
  MMP_EHIP = -5,        /* HIP runtime error; see mmp_last_hip_error() */
  MMP_EBUSY = -6,       /* server admission rejected (non-blocking submit) */
  MMP_ENOTFOUND = -7,   /* unknown server ticket or operand handle */
  MMP_ETIMEOUT = -8     /* mmp_wait timed out */
} mmp_status;

/* Word forms. */
enum {
  MMP_FORM_AUTO = 0,        /* planner picks the faster form for (p, shape) */
  MMP_FORM_FP64_WORDS = 1,  /* the paper's binary64 words on FP64 MFMA */
  MMP_FORM_INT8_WORDS = 2   /* signed 8-bit digits on INT8 MFMA, int32
                               accumulation, binary64 reduction/recombination */
};

/* The INT8 digit planes of one operand, made once by mmp_prepare_operand and
 * reused by INT8-form products: the fixed A of the unbalanced block-Wiedemann
 * benchmark of Section 4.1, whose decomposition the paper times apart from
 * the products.  Filled by the library; the caller owns the planes' memory. */
typedef struct {
  const int8_t *planes;   /* device; `digits` planes of outer x kp signed
                             base-256 digits (outer = rows of an A, cols of
                             a B), each in 1 KB blocks of 16 outer rows by
                             64 inner bytes; the layout is the library's */
  uint64_t p;             /* the modulus the entries were reduced for */
  int side;               /* 0: an A (rows x cols = m x k); 1: a B (k x n) */
  int digits;             /* ceil(bits(p) / 8) */
  int64_t rows, cols;     /* the shape of the matrix they were made from */
  int64_t kp;             /* inner dimension rounded up to a multiple of 64 */
} mmp_operand_t;

/* Options; a NULL mmp_opts* means all fields zero. */
typedef struct {
  int form;               /* MMP_FORM_* */
  int validate_entries;   /* 1: check every entry of A and B lies in [0, p)
                             and is integral before computing (MMP_ERANGE);
                             the call then waits for the check to finish */
  int tile;               /* 0: planner's tile; else a tile id from mmp_plan_t */
  int strict_fmod;        /* 1: every in-loop reduction is the full Alg. 1;
                             0: the planner may use the correction-free form
                             where its range check allows (see mmp_plan_t) */
  int64_t force_kblock;   /* 0: planner's k-block; else the number of k-terms
                             accumulated between reductions (<= the bound;
                             FP64 form: at most 16, or a multiple of 4 up to
                             2^26; INT8 form: a multiple of 64 up to
                             kblock_int8) */
  void *workspace;        /* optional caller-owned device workspace; when
                             NULL the library allocates stream-ordered memory
                             from the device's default pool.  Pass one (of at
                             least the queried size) to capture a call into a
                             HIP graph. */
  size_t workspace_bytes; /* size of workspace */
  int extended_block;     /* FP64 form, 1: accumulate over the whole signed
                             exact range [-2^t, 2^t] instead of [0, 2^t]: each
                             in-loop reduction maps the accumulator to
                             [-2^t, -2^t + 4p) (a biased Alg. 1 with the same
                             three operations), so a block may hold L terms
                             with L w + 4p - 1 <= 2^(t+1), about twice the
                             paper's lambda (project-derived bound; w is the
                             paper's per-term bound).  0: the paper's bound. */
  int splits;             /* split-K: 0 = planner's choice (used when a
                             product has too few output tiles for the chip
                             and a long k), 1 = never, > 1 = that many
                             k-ranges; their residues are added mod p */
  int centered_words;     /* FP64 form, 1: centered words (project-derived
                             variant of Alg. 4): each entry x is first mapped
                             to x - p when 2x > p, then split with
                             round-to-nearest quotients, so every word lies
                             within alpha/2 + 2 of zero and a word product is
                             about a quarter of the paper's bound; the
                             in-loop reduction rounds the quotient to nearest
                             (c = floor(x q + 1/2)), leaving |x| <= p/2 + 4,
                             and a block may hold L terms with
                             p/2 + 4 + L W <= 2^t (W: the product of the two
                             word bounds).  Exclusive with extended_block and
                             strict_fmod.  0: the paper's words. */
  int batch_launch;       /* mm_modp_batched, INT8-form products:
                             0 = one launch of the digit planes and one of
                             the digit GEMM for every 64 products, whatever
                             their digit counts, when the batch has two or
                             more; 1 = per digit count (planes per product,
                             then one GEMM per digit count and 16
                             products); 2 = the one-launch form always.
                             Other entry points: must be zero. */
  const mmp_operand_t *prepared_a; /* mm_modp_async only: A's digit planes
                             from mmp_prepare_operand (same p and shape);
                             the product then takes the
                             INT8 form and reads the planes instead of
                             digitising A (A itself is not read).  NULL:
                             none.  Other entry points return MMP_EINVAL
                             when it is set. */
  const mmp_operand_t *prepared_b; /* the same for B */
} mmp_opts;

/* What the planner decided for one product (mmp_plan fills it). */
typedef struct {
  uint64_t p;
  int u, v;               /* words of A and of B */
  int form;               /* MMP_FORM_FP64_WORDS or MMP_FORM_INT8_WORDS */
  uint64_t alpha, beta;   /* ceil(p^(1/u)), ceil(p^(1/v)) (FP64 form) */
  int64_t lambda;         /* the paper's block size: eq. lambda-sw for (1,1),
                             eq. cAcB otherwise (FP64 form) */
  int64_t kblock;         /* k-terms accumulated between reductions (<= lambda) */
  int slots;              /* MFMA k-slots that hold one k-block (>= kblock;
                             4, 8 or 16 with the excess slots holding zeros,
                             or equal to kblock, a multiple of 4) */
  int lazy;               /* 1: in-loop reductions omit Alg. 1's corrections
                             (result in [-p, 2p), or [-2^t, -2^t + 4p) when
                             biased); the final one is complete */
  int extended;           /* 1: the extended block bound (mmp_opts) is used */
  int tile;               /* kernel tile id */
  int bm, bn, bk;         /* workgroup tile (rows, cols, k-slots per stage) */
  int digits_a, digits_b; /* INT8 form: signed base-256 digits per operand */
  int64_t kblock_int8;    /* INT8 form: k-terms per int32 accumulation block */
  double q;               /* fl(1/p) */
  double est_seconds;     /* planner's cost-model estimate (0 if unknown) */
  int splits;             /* split-K k-ranges (1: none) */
  size_t workspace_bytes; /* device workspace the call needs */
  int centered;           /* 1: centered words and the round-to-nearest
                             in-loop reduction (mmp_opts.centered_words) */
  int biased;             /* 1: the correction-free in-loop reduction is the
                             biased one, c = floor(x q + K) with
                             K = floor(2^t / p) - 1, which leaves the
                             accumulator in [-2^t, -2^t + 4p): always with
                             extended, and under the paper's bound when a
                             block of kblock <= lambda terms started in
                             [-p, 2p) could pass 2^t but one started there
                             cannot (e.g. (2,2) at 50 bits: kblock =
                             lambda = 7) */
} mmp_plan_t;

/* One product of a batch. */
typedef struct {
  uint64_t p;
  int u, v;               /* 0, 0: planner's choice */
  int64_t m, n, k;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double *C;
  int64_t ldc;
} mmp_job;

/* ---------------------------------------------------------------- core */

/* C = A B mod p, synchronous (returns after C is written), null stream,
 * contiguous matrices (lda = k, ldb = n, ldc = n).  u = v = 0 lets the
 * planner pick the words; otherwise 1 <= u, v <= 4 with u v <= 8.
 * Defined by Section 1 eq. goal; computed by the method of Section 3.2. */
int mm_modp(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k,
            const double *A, const double *B, double *C);

/* Same product with options, strides and a stream; asynchronous.
   The FP64-word kernel addresses one stage of A (a tile's rows) and of B
   (16 rows) with 32-bit byte offsets: (bm - 1) lda + 16 and 16 ldb + bn
   doubles must stay below 2^28.  Beyond that an AUTO call (u = v = 0, no
   word-form option) takes the INT8-digit form, and a call that forces the
   FP64 form returns MMP_EINVAL before any device work.  Batched products
   return MMP_EINVAL; the server plans such a request in the INT8 form. */
int mm_modp_async(const mmp_opts *opts, uint64_t p, int u, int v, int64_t m,
                  int64_t n, int64_t k, const double *A, int64_t lda,
                  const double *B, int64_t ldb, double *C, int64_t ldc,
                  void *stream);

/* The same product for callers that cannot allocate: code under HIP graph
 * capture, serving loops that must not touch the allocator, harnesses that
 * forbid it.  It calls no allocation routine.  Its workspace (digit planes
 * of the INT8 form, split-K residues) is a library-owned device array of
 * MMP_STATIC_SCRATCH_BYTES per device, held from the library's first use of
 * this entry point on that device until the process ends; the plan is the
 * one mm_modp_async makes.  MMP_ENOMEM when that plan needs more workspace
 * than the array holds (e.g. the INT8 form of 4096^3 at 5 or more digits:
 * pass a smaller product, fewer split-K ranges or FP64 words);
 * MMP_EINVAL when opts carries a workspace or asks for validate_entries.
 * Every call on one device shares that device's array: calls that overlap
 * in time on one device (concurrent streams or threads) race; order them
 * on one stream.  Nothing in the array needs to start at zero. */
#define MMP_STATIC_SCRATCH_BYTES (256u << 20)
int mm_modp_static(const mmp_opts *opts, uint64_t p, int u, int v, int64_t m,
                   int64_t n, int64_t k, const double *A, int64_t lda,
                   const double *B, int64_t ldb, double *C, int64_t ldc,
                   void *stream);

/* Device bytes of one operand's digit planes (0 for invalid arguments):
 * digits x outer16 x kp, with outer16 the rows of an A (side 0) or cols of a
 * B (side 1) rounded up to 16 and kp the inner dimension rounded up to 64. */
size_t mmp_operand_bytes(uint64_t p, int side, int64_t rows, int64_t cols);

/* Writes the signed base-256 digit planes of M (entries in [0, p), row
 * stride ld) into the caller's device buffer `planes` (at least
 * mmp_operand_bytes) on `stream`, and fills *out to describe them; pass
 * out through mmp_opts.prepared_a (side 0) or prepared_b (side 1).  The
 * digits are those the INT8 form makes per call (the multiword split of
 * Section 3.1 with 8-bit words, the low-precision words of Section 6).
 * Asynchronous; `planes` must stay valid and unchanged while products use
 * it.  MMP_EINVAL for bad arguments, a buffer too small or one that
 * overlaps M. */
int mmp_prepare_operand(uint64_t p, int side, const double *M, int64_t rows,
                        int64_t cols, int64_t ld, void *planes,
                        size_t planes_bytes, mmp_operand_t *out,
                        void *stream);

/* ---------------------------------------------------------------- batches */

/* count independent products C_i = A_i B_i mod p_i (each job with its own
 * shape, modulus and words), enqueued on one stream.  Products that share a
 * kernel configuration run in one launch (up to 16 per launch); no host
 * synchronisation happens unless validate_entries is set, so with a caller
 * workspace of mmp_workspace_batched() bytes the call can be captured into a
 * HIP graph.  The batched block products follow the paper's closing
 * perspective (Section 6).  Outputs must not overlap each other. */
int mm_modp_batched(const mmp_job *jobs, int count, const mmp_opts *opts,
                    void *stream);

/* Device workspace mm_modp_batched needs for these jobs and options (0 if the
 * jobs are invalid or need none). */
size_t mmp_workspace_batched(const mmp_job *jobs, int count,
                             const mmp_opts *opts);

/* Multi-modular product: C[i] = A B mod primes[i] for i < nprimes, for one
 * integer pair A (m x k), B (k x n) of uint64 entries below 2^entry_bits
 * (1 <= entry_bits <= 62; DEVICE pointers, row-major, leading dimensions
 * lda, ldb).  primes is a HOST array of moduli in [5, 2^52); C is a HOST
 * array of nprimes DEVICE pointers to m x n binary64 outputs (leading
 * dimension ldc, pairwise disjoint).  This is the multimodular setting the
 * paper compares against (Section 5.2): with k within one exact int32 block
 * the integer product's digit-weight sums are formed once on the INT8 matrix
 * cores and every modulus reduces them (one GEMM launch for up to 64
 * moduli); otherwise A and B are reduced mod each p on the device and the
 * products run as a batch.  validate_entries checks the entry bound
 * (MMP_ERANGE).  Capturable into a graph with a caller workspace of
 * mmp_workspace_crt() bytes. */
int mm_modp_crt(const mmp_opts *opts, const uint64_t *A, int64_t lda,
                const uint64_t *B, int64_t ldb, int64_t m, int64_t n,
                int64_t k, int entry_bits, const uint64_t *primes,
                int nprimes, double *const *C, int64_t ldc, void *stream);

/* Device workspace mm_modp_crt needs (0 for invalid arguments). */
size_t mmp_workspace_crt(int64_t m, int64_t n, int64_t k, int entry_bits,
                         int nprimes, const mmp_opts *opts);

/* Chinese remainder reconstruction (Section 5.2): for every entry (i, j) of
 * nmoduli residue matrices, the unique integer X in [0, M), M = moduli[0]
 * ... moduli[nmoduli - 1], with X = C[t][i][j] mod moduli[t] for every t.
 * X is the integer product A B that mm_modp_crt's residues come from when M
 * exceeds its entries (eq. CRT2: M > k (2^entry_bits - 1)^2).
 *   C: HOST array of nmoduli DEVICE pointers to m x n binary64 residues
 *      (integers in [0, moduli[t]), leading dimension ldc);
 *   moduli: HOST array, 1 <= nmoduli <= 64, pairwise coprime, each in
 *      [2, 2^52 / 3] (the range where Alg. 2 is exact for factors below the
 *      modulus, Prop. Joris);
 *   out: DEVICE, X as `limbs` little-endian 64-bit words in planes: word w of
 *      entry (i, j) at out[(w m + i) ldo + j]; limbs must hold M - 1.
 * Computed on the device: Garner's mixed-radix digits in binary64 modular
 * arithmetic (Alg. 1, Alg. 2), then Horner into the limbs.  Asynchronous on
 * `stream`; MMP_EINVAL for bad arguments, before any launch. */
int mmp_crt_reconstruct(const double *const *C, int64_t ldc,
                        const uint64_t *moduli, int nmoduli, int64_t m,
                        int64_t n, uint64_t *out, int64_t ldo, int limbs,
                        void *stream);

/* ---------------------------------------------------------------- serving */

/* A request server on one device: products of mixed shapes and moduli are
 * submitted as they arrive and served with continuous batching.  A
 * scheduler thread admits queued requests in arrival order while a request
 * slot is free and the device footprint in flight (mmp_footprint of each
 * admitted request: operands, result and word or digit copies, per the
 * storage cost of Section 3.3) stays within hbm_budget; all requests
 * admitted in one scheduling step are launched together (products sharing a
 * kernel configuration in one launch) on the least busy of 4 streams, so
 * requests that arrive while others run start beside them and their work
 * overlaps on the device.  Results are identical to single calls: every
 * product is exact. */
typedef struct mmp_server mmp_server;

enum {
  MMP_SERVER_DRY_RUN = 1,  /* no device work: each batch completes after the
                              planner's time estimate; exercises admission,
                              queueing and latency accounting only (outputs
                              are not written) */
  MMP_SERVER_FAIL_LAUNCHES = 2, /* testing aid: every batch fails at launch
                              with MMP_ENOMEM before any device work, so the
                              failure path (requests completed with that
                              status, waiters woken) runs on the host */
  MMP_SUBMIT_NOQUEUE = 1   /* reject with MMP_EBUSY instead of queueing when
                              the request cannot be admitted at once */
};

typedef struct {
  int64_t submitted, completed, failed, rejected;
  int64_t launches, max_batch;  /* batches launched, largest batch */
  int64_t queued, running;      /* requests waiting / in flight now */
  size_t used_bytes, peak_used_bytes, resident_bytes;
  int64_t max_inflight;         /* most batches in flight at once */
  int64_t max_running;          /* most requests in flight at once */
} mmp_server_stats_t;

/* Starts a server on `device` (flags: 0, MMP_SERVER_DRY_RUN and/or
 * MMP_SERVER_FAIL_LAUNCHES). */
int mmp_server_create(mmp_server **out, int device, size_t hbm_budget,
                      int max_slots, int flags);

/* Finishes all queued and running requests, then frees the server, its
 * streams and resident operands. */
int mmp_server_destroy(mmp_server *srv);

/* Keeps the INT8 digit planes of a caller-owned matrix resident: side 0
 * registers an A operand (rows x cols = m x k), side 1 a B operand (k x n),
 * for modulus p.  A later request whose A (or B) has this pointer, shape,
 * leading dimension and modulus skips digitising it (the paper's setting of
 * a fixed A reused across products, Section 4.1); an AUTO request (u = v =
 * 0) with a resident operand takes the INT8 form.  The planes count against
 * the budget until mmp_unregister_operand.  The matrix must not change while
 * registered, and device work that writes it must have completed before
 * this call.  Synchronous. */
int mmp_register_operand(mmp_server *srv, const double *M, int64_t rows,
                         int64_t cols, int64_t ld, uint64_t p, int side,
                         uint64_t *handle);

/* Waits for requests that use the operand, then frees its planes. */
int mmp_unregister_operand(mmp_server *srv, uint64_t handle);

/* Queues one product (non-blocking); *ticket identifies it.  MMP_ENOMEM if
 * its footprint can never fit the budget; with MMP_SUBMIT_NOQUEUE,
 * MMP_EBUSY when it cannot be admitted immediately.  The job's buffers must
 * stay valid until the ticket is reported done.  The server's streams are
 * not ordered after any caller stream: device work that writes A, B or C
 * must have completed before mmp_submit is called (e.g. by synchronising
 * the stream that ran it), and C must not be touched until the ticket is
 * reported done. */
int mmp_submit(mmp_server *srv, const mmp_job *job, int flags,
               uint64_t *ticket);

/* mmp_submit, ordered after the work already queued on the caller's
 * `stream` (a hipStream_t as void*): an event recorded there at submission
 * is waited for on the device by the server's launch stream, so A, B and C
 * may still be in production on `stream` when this is called.  The host
 * does not block.  NULL is the null stream, as everywhere in this library.
 * In dry-run mode the stream is ignored. */
int mmp_submit_after(mmp_server *srv, const mmp_job *job, int flags,
                     void *stream, uint64_t *ticket);

/* *done = 1 when the request has completed; then *status is its result
 * code and *latency_s the time from submission to completion, and the
 * ticket is forgotten (a second poll returns MMP_ENOTFOUND). */
int mmp_poll(mmp_server *srv, uint64_t ticket, int *done, int *status,
             double *latency_s);

/* Blocks until the request completes (timeout_s < 0: no limit), then reports
 * as mmp_poll does; MMP_ETIMEOUT if the time runs out first. */
int mmp_wait(mmp_server *srv, uint64_t ticket, double timeout_s, int *status,
             double *latency_s);

/* Counters and current occupancy. */
int mmp_server_stats(mmp_server *srv, mmp_server_stats_t *out);

/* ---------------------------------------------------------------- planning */

/* Fills *out with the plan mm_modp_async would use (host-only; touches no
 * device).  Word counts and block size follow Section 3.3 (Table
 * tab.summary and the bitsize ranges after it) and Prop. UVMW. */
int mmp_plan(uint64_t p, int u, int v, int64_t m, int64_t n, int64_t k,
             const mmp_opts *opts, mmp_plan_t *out);

/* Autotuner: times every candidate plan for this product shape on the
 * current device (each admissible (u, v) with each tile and its block under
 * the paper's bound, or the extended one if opts allows it, and the INT8-digit
 * form) on scratch operands, and caches the fastest for the class of
 * products with the same bitsize of p and the same ceil(log2) of m, n and k.
 * Later AUTO plans (u = v = 0, no forced tile or block) of that class use it.
 * *best receives the resulting plan, *tried the number of candidates timed.
 * Synchronous; allocates 8 (mk + kn + mn) bytes of scratch. */
int mmp_autotune(uint64_t p, int64_t m, int64_t n, int64_t k,
                 const mmp_opts *opts, mmp_plan_t *best, int *tried);

/* Tuning cache: forget all entries; write or read them as JSON (load returns
 * the number of entries read or a negative status). */
int mmp_tune_cache_clear(void);
int mmp_tune_cache_save(const char *path);
int mmp_tune_cache_load(const char *path);

/* The exact int32 block of the INT8-digit form (the low-precision words of
 * Section 6; the block length plays the part of the paper's lambda, Section
 * 2.2).  The digit GEMM sees each entry as an integer x' in [lo, hi] written
 * with `digits` signed base-256 digits in [-128, 127]; one k-term adds
 * sum_{i+j=s} a_i b_j to the int32 accumulator of digit weight 256^s.
 * term_max and term_min are the exact extremes of that sum over all pairs of
 * entries (any weight s), reached by the entries witness_max = (a, b) and
 * witness_min at weights weight_max and weight_min; kblock is the largest
 * multiple of 64 with kblock * term_max <= 2^31 - 1 and
 * kblock * (-term_min) <= 2^31, the k-terms the GEMM accumulates between
 * folds (mmp_plan_t.kblock_int8).  Host-only. */
typedef struct {
  int digits;
  int weight_max, weight_min;
  int64_t lo, hi;
  int64_t term_max, term_min;
  int64_t witness_max[2], witness_min[2];
  int64_t kblock;
} mmp_int8_bound_t;

/* Residues mod p (entry_bits = 0): x' = x, or x - p when x exceeds
 * 127 (256^D - 1) / 255, with D = ceil(bitsize(p) / 8).  Integers of
 * mm_modp_crt (p = 0, 1 <= entry_bits <= 62): x' = x in [0, 2^entry_bits),
 * with the fewest digits that hold them.  MMP_EINVAL otherwise. */
int mmp_int8_bound(uint64_t p, int entry_bits, mmp_int8_bound_t *out);

/* The same for any interval lo <= hi of values that `digits` (1..8) signed
 * digits hold, [-128 (256^D - 1) / 255, 127 (256^D - 1) / 255] (digits = 8:
 * within int64).  MMP_EINVAL otherwise. */
int mmp_int8_interval_bound(int digits, int64_t lo, int64_t hi,
                            mmp_int8_bound_t *out);

/* Device bytes a job occupies: its operands and result (8 (mk + kn + mn))
 * plus its word copies (FP64 words: 8 (u mk + v kn); INT8 digits: the
 * digit planes as the library lays them out, about da mk + db kn with rows
 * rounded up to 16 and k to 64), per the storage cost of Section 3.3. */
size_t mmp_footprint(const mmp_job *job, const mmp_plan_t *plan);

/* Static description of a status code (never NULL). */
const char *mmp_strerror(int status);

/* The hipError_t of the last MMP_EHIP on this thread (0 if none). */
int mmp_last_hip_error(void);

/* ---------------------------------------------------------------- timers */

/* Per-phase kernel time.  When enabled, every launch the library makes is
 * bracketed by a HIP event pair on its stream; mmp_timers_read waits for the
 * recorded events and reports, per phase ("fp64_words", "int8_digitize" for
 * both operands in one launch, "int8_digitize_a" or "int8_digitize_b" for
 * one, "int8_gemm", "int8_gemm_persistent", ...), the number of launches and
 * their summed device time.  This measures the paper's time breakdown
 * (Section 4.2.1) on the device instead of on the host. */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
} mmp_timer;

/* on = 1 starts recording, 0 stops (already recorded pairs are kept). */
int mmp_timers_enable(int on);

/* Copies up to cap phase sums into out (cap = 0: only count) and returns the
 * number of phases; reset = 1 clears the sums afterwards.  Blocks until the
 * recorded events have completed. */
int mmp_timers_read(mmp_timer *out, int cap, int reset);

#ifdef __cplusplus
}
#endif

#endif /* MMP_H */
