/*
 * nttmi: exact digital circular convolution modulo a prime m through a
 * number-theoretic transform whose root of unity is a power of two, on AMD
 * MI355X (gfx950).
 *
 * Method: S. S. Chandra, "Fast Digital Convolutions using Bit-Shifts"
 * (arXiv:1005.1497).  The circular convolution of Eq. 1 is computed with the
 * convolution theorem (Sec. I): forward transform of both sequences (Eq. 2),
 * pointwise product modulo m, inverse transform with the factor N^-1 (Eq. 3).
 * The root of unity of order N is a power of two 2^k modulo a Rader prime m
 * (a prime factor of a Fermat number, Prop. 2; Table 1), so the transform
 * coefficients are the "harmonics" 2^e mod m of the digital circle (Eq. 5).
 *
 * C ABI.  No C++ types and no exceptions cross this boundary.  All pointers
 * named f, g, h, x, X are DEVICE pointers to little-endian unsigned words of
 * elem_bits bits, owned by the caller; the library keeps none of them after
 * a call returns (the served-form calls ntt_copy_batch and ntt_server_* state
 * their own host or device pointers).  `stream` is a hipStream_t (NULL = the
 * null stream).
 *
 * Results are exact residues in canonical form [0, m) (Appendix A).  Inputs
 * may hold any elem_bits-bit value; it is read modulo m.
 *
 * Every call validates its arguments on the host before any device work and
 * returns a status; on an argument error nothing is enqueued and no memory is
 * touched.  On success the work is enqueued on `stream` and the call returns
 * without waiting; device faults surface at the caller's next
 * synchronisation.  The library owns per-plan device tables (powers of the
 * root) and workspaces in process-wide caches, created on first use and freed
 * by ntt_release_caches().  Calls are thread-safe; calls that overlap on the
 * same stream are ordered by the stream.
 */
#ifndef NTTMI_H
#define NTTMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NTT_OK = 0,
    NTT_E_ARG = 1,          /* null pointer, bad elem_bits, bad descriptor, partial overlap */
    NTT_E_MODULUS = 2,      /* m not prime, order of 2 mod m not a power of two, or m too
                               wide for elem_bits (32-bit words: m < 2^24) */
    NTT_E_LENGTH = 3,       /* N = 2^log2n does not divide the order of 2 mod m */
    NTT_E_ROOT = 4,         /* root is not of exact order N modulo m */
    NTT_E_RANGE = 5,        /* an operand >= m, only with NTT_FLAG_CHECK_RANGE */
    NTT_E_NOMEM = 6,        /* device or host allocation failed */
    NTT_E_DEVICE = 7,       /* a HIP runtime call or kernel launch failed */
    NTT_E_UNSUPPORTED = 8,  /* a valid request the library does not implement (64-bit
                               words: m >= 2^46; lengths above 2^22) */
    NTT_E_SINGULAR = 9,     /* conv_deconvolve: a spectral coefficient of the divisor
                               is zero, so no unique quotient exists */
    NTT_E_TIMEOUT = 10,     /* ntt_server_wait: the time limit passed first */
    NTT_E_NOPLAN = 11       /* conv_circular_noalloc: the plan of (m, N, root) has not
                               been built on this device by an earlier call */
} ntt_status;

/* Flags (bitwise OR). */
#define NTT_FLAG_CHECK_RANGE   0x1u  /* reject operands >= m with NTT_E_RANGE; this
                                        reads them back and synchronises the stream */
#define NTT_FLAG_PER_ITEM      0x2u  /* conv_batched: one launch sequence per item
                                        (the unfused reference form) */
#define NTT_FLAG_PER_CLASS     0x4u  /* conv_batched: one launch per length class
                                        instead of one persistent launch */
#define NTT_FLAG_AUTOTUNE      0x8u  /* conv_batched: time the candidate forms of this
                                        batch (one persistent launch or one launch per
                                        length; per length: LDS tile of 256 threads or
                                        of one wave, fused kernel at full or one-per-CU
                                        occupancy, or the unfused four-step launches
                                        with 512- or 256-thread workgroups),
                                        keep the fastest for every later batch of the
                                        same shape (lengths, item counts rounded down to
                                        powers of two, m, word width, device), and run
                                        it.  Synchronises the stream; not for use while
                                        the stream is being captured into a graph */
#define NTT_FLAG_EULER         0x10u /* the Euler (Pollard) form of Sec. I, Eq. 6: any
                                        prime m (not only those of which 2 is a
                                        lambda-root) with N | m - 1, and a root of exact
                                        order N that need not be a power of two
                                        (ntt_euler_root gives one).  Lengths up to
                                        2^v, 2^v the largest power of two dividing m - 1
                                        (ntt_max_log2n).  conv_batched:
                                        root_log2order <= v */
#define NTT_FLAG_TRANSIENT     0x20u /* conv_batched: the descriptor is used once (a
                                        served batch).  It goes into a per-stream ring
                                        of pinned host slots that the kernels read
                                        directly (no copy), instead of the
                                        content-addressed descriptor cache, so a stream of distinct
                                        batches never evicts that cache (which
                                        synchronises the device).  Ignored while the
                                        stream is being captured (captured kernels need
                                        descriptors that later calls do not overwrite) */

/* Batch of independent convolutions of uneven power-of-two lengths.
 * Item i has length N_i = 2^log2n[i] and occupies elements
 * [offset[i], offset[i] + N_i) of each of f, g and h.  Items must not overlap
 * one another.  Both arrays are HOST memory and are read during the call only. */
typedef struct {
    uint32_t        count;   /* number of items (0 is allowed: nothing to do) */
    const uint8_t  *log2n;   /* [count] log2 of each length */
    const uint64_t *offset;  /* [count] element offset of each item */
} ntt_batch_desc;

/* Forward transform of Eq. 2 with `root` in place of 2 (Eq. 2 is the case
 * N = N_Max, root = 2):  X(u) = < sum_t x(t) root^(u t) >_m, u = 0..N-1, in
 * natural order.  `batch` rows of N = 2^log2n contiguous elements each.
 * Requirements: m prime with ord_m(2) = nu a power of two (Sec. II, Prop. 2),
 * N | nu (Sec. I), root of exact order N (root^(N/2) = m - 1 for N >= 2,
 * root = 1 for N = 1).  In place (x == X) is allowed. */
ntt_status ntt_forward(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits,
                       const void *x, void *X, uint32_t batch, uint32_t flags,
                       void *stream);

/* Inverse transform of Eq. 3, including the factor N^-1 (the multiplicative
 * inverse of N modulo m, Appendix A):  x(t) = < N^-1 sum_u X(u) root^(-u t) >_m.
 * ntt_inverse(ntt_forward(x)) = x for x in [0, m).  Same requirements and
 * layout as ntt_forward; in place allowed. */
ntt_status ntt_inverse(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits,
                       const void *X, void *x, uint32_t batch, uint32_t flags,
                       void *stream);

/* Circular convolution of Eq. 1 of two length-N sequences:
 *   h(j) = < sum_{k<N} f(k) g(j - k mod N) >_m
 * computed by the convolution theorem with the given root.  h may equal f or g
 * (in place); partial overlap is NTT_E_ARG. */
ntt_status conv_circular(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits,
                         const void *f, const void *g, void *h, uint32_t flags,
                         void *stream);

/* conv_circular for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * result and arguments as conv_circular.  The call allocates no device or
 * host memory and never synchronises: lengths above 2^12 keep their 2N
 * scratch words in a static device array of the library (4 MiB per device,
 * held until the process ends) instead of a per-stream workspace; shorter
 * lengths need no scratch.  The first such call on a device looks up the
 * array's device address, which makes the HIP runtime load the code object
 * that holds it (a one-time set-up per device, done by the runtime).
 *   - 2 N (elem_bits / 8) <= 4 MiB: N <= 2^19 with 32-bit words, N <= 2^18
 *     with 64-bit words; longer: NTT_E_UNSUPPORTED, nothing enqueued.
 *   - The plan of (m, N, root) (its device tables) must already exist on the
 *     current device, built by an earlier allocating call with the same m, N
 *     and root (conv_circular, ntt_forward, ntt_inverse, conv_batched for a
 *     root of that order); otherwise NTT_E_NOPLAN, nothing enqueued.
 *   - NTT_FLAG_CHECK_RANGE is refused (NTT_E_UNSUPPORTED): it reads back.
 * Every call on a device shares that device's one scratch array, which keeps
 * the last call's contents (each call writes its scratch before reading it):
 * calls that overlap in time on one device (on different streams, or from
 * several host threads without ordering) race on it and give undefined
 * results.  Order them, for example on one stream. */
ntt_status conv_circular_noalloc(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits,
                                 const void *f, const void *g, void *h, uint32_t flags,
                                 void *stream);

/* A batch of independent circular convolutions of uneven power-of-two lengths
 * (see ntt_batch_desc), all modulo the same m.  `root` has exact order
 * 2^root_log2order; item i uses root^(2^(root_log2order - log2n[i])), of
 * exact order N_i, so log2n[i] <= root_log2order is required.  The usual choice
 * is root = 2 and root_log2order = log2(ord_m(2)).  Default form:
 *   - one length: lengths up to 2^12 run the LDS kernel (several items per
 *     workgroup); longer lengths run the persistent fused kernel (one item per
 *     workgroup at a time, from a per-stream work queue), except that a batch
 *     whose items are back to back and number fewer than two thirds of that
 *     kernel's resident workgroups runs the multi-launch four-step form,
 *     whose phases spread every item over the chip;
 *   - several lengths: one persistent launch covers every length up to 2^19
 *     (32-bit words) or 2^18 (64-bit words), except that a batch with fewer
 *     tasks than two thirds of that kernel's resident workgroups, whose items
 *     of each length above 2^12 lie back to back, runs one launch per length
 *     (each as above); longer lengths run one launch per length.
 * A form tuned with NTT_FLAG_AUTOTUNE for the batch's shape replaces the
 * default.  Every form gives the same result.  A call is capturable into a
 * HIP graph on a stream once a call with the same batch shape (lengths, item
 * counts, layout) has run on that stream: its plans, workspaces, work queue
 * and any tuning are then in place.  The captured kernels keep that stream's
 * workspace and work queue: replay the graph on that stream, or ordered with
 * every other use of it.  A workspace that a later call outgrows is retired,
 * not freed, so the graph stays valid until ntt_release_caches.  f, g and h
 * may be device memory or pinned host memory (hipHostMalloc, passed at the
 * address hipHostGetDevicePointer gives): the kernels then load and store them
 * over the host link,
 * with no copies (ntt_server_create_host works so); the scratch stays on the
 * device. */
ntt_status conv_batched(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits,
                        const ntt_batch_desc *d, const void *f, const void *g, void *h,
                        uint32_t flags, void *stream);

/* Exact deconvolution (division filtering): a prime modulus makes every
 * nonzero coefficient invertible (Sec. III-A), so f * g = h (Eq. 1) is solved
 * for g by the convolution theorem read backwards (Sec. I):
 *     g = inverse( forward(h) / forward(f) ),
 * the spectral quotients formed with Fermat inverses F(u)^(m-2).  `batch` rows
 * of N = 2^log2n contiguous elements; row r of g solves row r of f and h.
 * Same requirements on m, N and root as conv_circular (NTT_FLAG_EULER
 * applies).  Returns NTT_E_SINGULAR when some forward(f) coefficient of some
 * row is zero (g is then unspecified).  Synchronises the stream (it reads the
 * singular flag back), so it is refused (NTT_E_UNSUPPORTED, nothing enqueued)
 * while the stream is being captured.  g may equal h (in place); partial
 * overlap is NTT_E_ARG. */
ntt_status conv_deconvolve(uint64_t m, uint32_t log2n, uint64_t root, uint32_t elem_bits,
                           const void *f, const void *h, void *g, uint32_t batch,
                           uint32_t flags, void *stream);

/* Exact integer circular convolution (Eq. 1 without the modulus) by residue
 * number arithmetic: the convolution modulo the Rader prime 13631489 =
 * 13 * 2^20 + 1 and modulo the Euler-form prime 7340033 = 7 * 2^20 + 1,
 * combined by the Chinese remainder theorem into the unique value in
 * [0, 13631489 * 7340033) (about 1.0006e14, 2^46.5).  f and g: `batch` rows of
 * N = 2^log2n uint32 words, read as non-negative integers; h: uint64 words.
 * h equals the true integer convolution whenever every true value is below
 * that product (e.g. N <= 2^16 with operands below 2^15); otherwise it is the
 * true value modulo the product.  log2n <= 19.  h may not overlap f or g.
 * Asynchronous; capturable after a first call on the stream. */
ntt_status conv_crt(uint32_t log2n, const void *f, const void *g, void *h, uint32_t batch,
                    uint32_t flags, void *stream);

/* Two-dimensional circular convolution of R x C arrays (row-major, R = 2^log2r
 * rows, C = 2^log2c columns), the multi-dimensional form of Eq. 1:
 *   h(i, j) = < sum_{k, l} f(k, l) g((i - k) mod R, (j - l) mod C) >_m,
 * computed with row transforms, a transpose and column transforms (each
 * dimension by Eq. 2 with its own root of exact order R or C), the pointwise
 * product, and the inverses (Eq. 3, with R^-1 and C^-1).  Same requirements on
 * m and the roots as conv_circular, per dimension (NTT_FLAG_EULER applies);
 * R C <= 2^31.  h may equal f or g; partial overlap is NTT_E_ARG.
 * Asynchronous. */
ntt_status conv2d_circular(uint64_t m, uint32_t log2r, uint32_t log2c, uint64_t root_r, uint64_t root_c,
                           uint32_t elem_bits, const void *f, const void *g, void *h, uint32_t flags,
                           void *stream);

/* The default root for length 2^log2n: 2^(nu / N), nu = ord_m(2) (the harmonic
 * of the digital circle of Eq. 5 that has exact order N).  Writes it to *root. */
ntt_status ntt_default_root(uint64_t m, uint32_t log2n, uint64_t *root);

/* log2 of ord_m(2) for a valid modulus (Prop. 2), written to *log2_nu. */
ntt_status ntt_modulus_order(uint64_t m, uint32_t *log2_nu);

/* Euler form (NTT_FLAG_EULER): for a prime m, the largest n with 2^n | m - 1,
 * written to *log2n (NTT_E_MODULUS when m is not prime). */
ntt_status ntt_max_log2n(uint64_t m, uint32_t *log2n);

/* Euler form: a root of exact order 2^log2n modulo the prime m (requires
 * 2^log2n | m - 1): z^((m - 1) / 2^log2n) for the smallest quadratic
 * non-residue z.  Writes it to *root. */
ntt_status ntt_euler_root(uint64_t m, uint32_t log2n, uint64_t *root);

/* Staging helper for the served form (plumbing, no arithmetic of the method):
 * enqueues count asynchronous copies dst[i] <- src[i] of bytes[i] bytes on
 * `stream`, in index order, with hipMemcpyDefault (each side device memory or
 * pinned host memory), so that a batch of requests is uploaded or downloaded
 * in one call rather than one per request.  dst, src and bytes are host arrays
 * of count entries owned by the caller and read before the call returns; the
 * buffers they point to must stay valid until the stream has run the copies.
 * A zero-byte entry is skipped.  NTT_E_ARG: a null array with count > 0, or a
 * null pointer in an entry of non-zero size (nothing is enqueued then);
 * NTT_E_DEVICE: the runtime refused a copy (the copies before it stay
 * enqueued). */
ntt_status ntt_copy_batch(void *const *dst, const void *const *src, const uint64_t *bytes, uint32_t count,
                          void *stream);

/* Native served form (plumbing around conv_batched, no arithmetic of its own).
 * ntt_server_create: a server owns three device arenas of 2^arena_log2 words
 * (f, g, h; ntt_server_create_host keeps them in pinned host memory instead,
 * see there), a set of
 * non-blocking streams and one scheduler thread.  ntt_server_submit copies a
 * request's operands (host memory) into a pinned staging block and queues it;
 * the scheduler admits queued requests in arrival order while a buddy
 * allocator over the arenas has room (every request takes one slot of its
 * length, the same offset in all three arenas), at most max_batch requests
 * and max_batch_elems arena words per batch (one larger request still goes
 * alone), with at most max_inflight batches on the device; a batch is one
 * upload call, one conv_batched call (NTT_FLAG_TRANSIENT) and one download on
 * the next stream.  ntt_server_wait blocks until the request is done and copies
 * its result to host memory.  Requests use root^(2^(root_log2order - log2n)),
 * as in conv_batched. */
typedef struct ntt_server ntt_server;

/* Creates a server.  elem_bits, m, root and root_log2order as for conv_batched;
 * arena_log2 <= 28; streams in [1, 16]; max_batch >= 1; max_batch_elems 0 means
 * the whole arena; max_inflight >= 1.  Allocates the arenas and, per stream,
 * the scratch workspace the batch kernels may take (at most 1 GiB), on the
 * current device.  NTT_E_ARG, NTT_E_MODULUS, NTT_E_LENGTH, NTT_E_ROOT as for
 * conv_batched; NTT_E_NOMEM; NTT_E_DEVICE. */
ntt_status ntt_server_create(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits,
                             uint32_t arena_log2, uint32_t streams, uint32_t max_batch, uint64_t max_batch_elems,
                             uint32_t max_inflight, ntt_server **out);

/* A server whose arenas are pinned host memory that the batch kernels read
 * and write directly over the host link: a request takes its slot when it is
 * submitted or staged (the same offset in three host arenas, chunks of
 * 2^arena_log2 words, a new chunk when the others are full), submit copies f
 * and g into it, a batch is requests of one chunk run by one conv_batched call
 * with no copies before or after it, and ntt_server_wait copies the result
 * out of the slot and frees it.  The device holds only the batch kernels'
 * scratch.  For requests whose transfer time matters more than the kernels'
 * (the kernels then load operands at the host link's rate).  Arguments and
 * errors as for ntt_server_create; every other ntt_server_* call applies. */
ntt_status ntt_server_create_host(uint64_t m, uint64_t root, uint32_t root_log2order, uint32_t elem_bits,
                                  uint32_t arena_log2, uint32_t streams, uint32_t max_batch,
                                  uint64_t max_batch_elems, uint32_t max_inflight, ntt_server **out);

/* Queues the convolution of f and g (host arrays of 2^log2n words each, read
 * before the call returns) and writes its ticket.  NTT_E_LENGTH: log2n above
 * root_log2order or arena_log2; NTT_E_ARG: null pointer or a stopped server;
 * NTT_E_NOMEM: no pinned staging memory (or host arena chunk). */
ntt_status ntt_server_submit(ntt_server *srv, const void *f, const void *g, uint32_t log2n, uint64_t *ticket);

/* Zero-copy submission, first half: reserves a staging block for a request of
 * 2^log2n words without queueing it, and writes host pointers to its f and g
 * rows (pinned memory owned by the server) and its ticket.  Fill both rows,
 * then call ntt_server_submit_staged.  Errors as for ntt_server_submit. */
ntt_status ntt_server_stage(ntt_server *srv, uint32_t log2n, void **f, void **g, uint64_t *ticket);

/* Zero-copy submission, second half: queues a staged request (its arrival
 * time is now).  NTT_E_ARG: an unknown ticket or one already queued. */
ntt_status ntt_server_submit_staged(ntt_server *srv, uint64_t ticket);

/* Waits up to timeout_s seconds (negative: no limit) for the request, copies
 * its 2^log2n result words to h (host) and releases the ticket.  NTT_E_ARG: an
 * unknown ticket, a staged one never queued, or a ticket another thread is
 * waiting for at the same time; NTT_E_DEVICE: its batch failed (the ticket is
 * released); NTT_E_TIMEOUT: the time ran out (the ticket stays valid). */
ntt_status ntt_server_wait(ntt_server *srv, uint64_t ticket, void *h, double timeout_s);

/* Completed requests since creation or the last reset, the mean requests per
 * batch, and the p50 / p99 of submit-to-completion latency in milliseconds over
 * the last 2^20 completed requests (completion as the scheduler observes it).
 * reset != 0 clears them. */
ntt_status ntt_server_stats(ntt_server *srv, uint64_t *completed, double *mean_batch, double *p50_ms,
                            double *p99_ms, uint32_t reset);

/* Admission policy: requests of 2^solo_log2n words and more are launched as
 * batches of their own, never together with other requests (0: no such
 * limit; the default is 16).  In a batch with other items a long convolution
 * runs on a single workgroup and every request of that batch completes only
 * with it; alone it takes the four-step form, whose phases spread over the
 * chip.  Applies to requests admitted after the call.  NTT_E_ARG: null
 * server. */
ntt_status ntt_server_set_solo(ntt_server *srv, uint32_t solo_log2n);

/* Finishes every queued and running request, stops the thread and frees the
 * server.  Tickets not yet waited for are released.  No other call on the
 * server may run concurrently with it or follow it.  The other ntt_server_*
 * calls are safe from several threads at once. */
void ntt_server_destroy(ntt_server *srv);

/* Diagnostics: cumulative counts, since the library was loaded (all devices
 * and threads), of the launches it has made by form and of its descriptor
 * uploads.  Writes counts[k] for k < min(n, NTT_COUNT_SLOTS); counts is a
 * host array owned by the caller.  Lets a caller (the tests) see which form
 * a call actually took: read before and after the call and compare. */
enum {
    NTT_COUNT_SMALL = 0,         /* LDS convolution kernels (N <= 2^12) */
    NTT_COUNT_FOURSTEP = 1,      /* multi-launch four-step convolutions (one per launch sequence) */
    NTT_COUNT_FUSED = 2,         /* persistent fused kernels of one length */
    NTT_COUNT_MULTI = 3,         /* persistent launches over several lengths */
    NTT_COUNT_TRANSFORM = 4,     /* transform launch sequences (ntt_forward / ntt_inverse rows) */
    NTT_COUNT_DESC_CACHED = 5,   /* descriptors uploaded into the content-addressed cache */
    NTT_COUNT_DESC_RING = 6,     /* descriptors uploaded through a stream's staging ring */
    NTT_COUNT_DESC_EVICTED = 7,  /* cache entries freed when the cache was full */
    NTT_COUNT_QUEUE_CREATED = 8, /* per-stream work queues created */
    NTT_COUNT_SLOTS = 9
};
void ntt_launch_counts(uint64_t *counts, uint32_t n);

/* Static description of a status code. */
const char *ntt_status_string(ntt_status s);

/* Frees the workspaces, work queue and staging ring the library holds for
 * `stream` on the current device, after waiting for the stream.  Call it
 * before destroying a stream the library has used: otherwise they stay until
 * ntt_release_caches, and a later stream that receives the same handle would
 * share them with work still pending on the old one.  Other calls on the same
 * stream must not run concurrently, and graphs captured on it before must not
 * be replayed after it. */
void ntt_release_stream(void *stream);

/* Frees every cached plan, workspace, descriptor and staging slot (waits for
 * the device first).  No other call of this library may run concurrently, and
 * graphs captured before it must not be replayed after it. */
void ntt_release_caches(void);

#ifdef __cplusplus
}
#endif

#endif /* NTTMI_H */
