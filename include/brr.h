/*
 * brr.h -- C ABI of libbrr, batched ranged random integers on MI355X (gfx950).
 *
 * The operations follow Brackett-Rozinsky and Lemire, "Batched Ranged Random
 * Integer Generation": several bounded integers a_i in [0, b_i) are taken
 * from one 64-bit random word r by the multiply chain of Theorem 1,
 * (a_i, r) <- b_i (x) r for i = 1..k, and the batch is accepted when the
 * leftover satisfies r >= 2^64 mod (b_1 ... b_k) (Lemire's criterion on the
 * bound product; Algorithms 2 and 3, Sec. 5); otherwise it is rolled again.
 * Shuffles apply Algorithm 4 (Sec. 6) batch by batch.
 *
 * Word source and addressing (not fixed by the paper; identical in every
 * entry point): word c of instance `inst` under `seed` is one 64-bit half of
 * Philox4x32-10 with key (lo32 seed, hi32 seed) and counter
 * (lo32 c/2, hi32 c/2, lo32 inst, hi32 inst); even c is x0 | x1 << 32, odd c
 * is x2 | x3 << 32. Attempt a (0 = first) of group/batch s of an instance
 * with S groups/batches reads word c = a*S + s. Results are therefore a pure
 * function of (inputs, seed, inst, schedule), independent of launch shape.
 * Two other streams follow the same addressing: the 32-bit halves of these
 * words (L = 32: brr_dice32, BRR_WORDS_PHILOX32 schedules) and ChaCha20
 * words (brr_dice_chacha, BRR_WORDS_CHACHA20 schedules). The division form
 * of Sec. 2.1 (brr_dice_div, BRR_FORM_DIVISION steps) reads the same words
 * as the multiply chain and splits the same value differently.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device pointers (HIP device memory, aligned to
 *    their element size, else BRR_EINVAL; 16-byte alignment is fastest).
 *    Pointers named h_* and struct pointers are host pointers read during
 *    the call.
 *  - The caller owns every buffer. The library keeps no pointer after a call
 *    returns, except that a brr_plan remembers the last buffers it was bound
 *    to (it is re-bound on each call).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is the
 *    null stream). Host-checkable errors return at once with nothing
 *    enqueued. Errors only the device can see (a zero bound, a bound product
 *    above 2^64 in a dice stream) are recorded in a per-device status word
 *    that brr_sync_status() returns; the affected outputs are unspecified.
 *  - Thread safety: calls may come from several host threads; work on one
 *    stream is ordered, work on different streams may overlap. A brr_plan
 *    serialises the host calls made on it, and each of its runs is ordered
 *    after its previous run whatever stream either was enqueued on (the runs
 *    share the plan's scratch); brr_plan_destroy must not overlap another
 *    call on the same plan.
 */
#ifndef BRR_H
#define BRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BRR_OK = 0,
    BRR_EINVAL = 1,    /* bad argument: null pointer, k = 0, zero bound, m > n, bad schedule */
    BRR_EOVERFLOW = 2, /* a bound product above 2^64 (Theorem 1 needs prod b_i <= 2^64) */
    BRR_ENOMEM = 3,    /* the library could not allocate device scratch memory */
    BRR_EHIP = 4,      /* a HIP runtime call failed */
    BRR_EDEVICE = 5    /* no usable gfx950 device */
} brr_status;

/* ------------------------------------------------------------------------ */
/* Batch-size schedules (Sec. 6 full-shuffle procedure, Sec. 6.1 batch sizes) */
/* ------------------------------------------------------------------------ */

#define BRR_MAX_STEPS 16
#define BRR_MAX_K 20 /* 21 dice never fit: 21! > 2^64 */

/* How a batch turns its word into dice:
 * BRR_FORM_MULTIPLY -- the multiply chain of Theorem 1 (Algorithm 4);
 * BRR_FORM_DIVISION -- the division form of Sec. 2.1, the comparison of the
 *   paper's experiments (its naive batched shuffle): one value V below the
 *   falling product i (i-1) ... (i-k+1) by Lemire's method (Sec. 2) on the
 *   batch's words, the die for bound i - l being the l-th successive
 *   remainder (V mod i first, then V div i continues); u0 is not used. */
#define BRR_FORM_MULTIPLY 0u
#define BRR_FORM_DIVISION 1u

/* While more than n_above elements remain to be shuffled, roll batches of k
 * dice in the given form; u0 is the initial upper bound on the batch's bound
 * product (Algorithm 4's u; 0 = none known, compare against the exact
 * product). A schedule's upper bounds only decide how often the exact
 * product is formed; they never change an output. Both forms read the same
 * words (the acceptance test is the same), so they differ only in the digits. */
typedef struct {
    uint64_t n_above;
    uint32_t k;
    uint32_t form; /* BRR_FORM_* (any other value: BRR_EINVAL) */
    uint64_t u0;
} brr_step;

/* The word stream every batch of a schedule reads (word c of instance inst):
 * BRR_WORDS_PHILOX64 -- the 64-bit Philox words of brr_dice;
 * BRR_WORDS_PHILOX32 -- their 32-bit halves, word c = half c mod 2 (low
 *   first) of 64-bit word c/2, with the chain and Lemire's threshold at
 *   L = 32 (Theorem 1 holds for any L, Sec. 4): every batch product at most
 *   2^32, multiply form only (the batch sizes of Table 2's L = 32 column);
 * BRR_WORDS_CHACHA20 -- the ChaCha20 words of brr_dice_chacha (the paper's
 *   slow generator, Sec. 7). */
#define BRR_WORDS_PHILOX64 0u
#define BRR_WORDS_PHILOX32 1u
#define BRR_WORDS_CHACHA20 2u

/* Steps run in order with non-increasing n_above. With tail = 1, when more
 * than one element remains after the last step, one batch of (i - 1) dice
 * bounded by u_tail finishes the shuffle (the last batch of Sec. 6; always
 * in the multiply form). words: BRR_WORDS_* (0 = Philox 64-bit words, what
 * every schedule-filling function sets unless stated otherwise); reserved
 * must be 0. */
typedef struct {
    uint32_t nsteps;
    uint32_t tail;
    uint64_t u_tail;
    brr_step step[BRR_MAX_STEPS];
    uint32_t words;
    uint32_t reserved;
} brr_schedule;

/* Fills *out with one of the paper's schedules (Sec. 7, Appendix A):
 * max_k = 6: shuffle_6 -- one die above 2^30 elements, then batches of 2, 3,
 *            4, 5, 6 dice at or below 2^30, 2^19, 2^14, 2^11, 2^9 elements
 *            with bounds 2^60, 2^57, 2^56, 2^55, 2^54, and a last batch of at
 *            most 5 dice bounded by 720;
 * max_k = 2: at most two dice (one die above 2^30, pairs bounded by 2^60,
 *            the same last-batch rule);
 * max_k = 1: the unbatched shuffle, one die per word.
 * Returns BRR_EINVAL for any other max_k or a null out. */
brr_status brr_schedule_paper(int max_k, brr_schedule *out);

/* Fills *out with the greedy largest-batch schedule (KMAX): while i elements
 * remain, batches of the largest k <= kcap whose product i (i-1) ... (i-k+1)
 * is at most 2^64 (the limit of Theorem 1 for 64-bit words). With N_k the
 * largest n whose k-th falling power is at most 2^64 (N_2 = 2^32,
 * N_3 = 2642246, N_4 = 65537, N_5 = 7133, N_6 = 1627, N_7 = 568, N_8 = 259),
 * step k runs while more than N_{k+1} elements remain, guarded by
 * N_k^(falling k); batches of kcap dice run while more than kcap - 1
 * elements remain, and a last batch (exact product) ends the shuffle. Large
 * batches reject more often (up to half the words near the top of a step);
 * the schedule is for comparison with the cost-model schedules.
 * 1 <= kcap <= 16, else BRR_EINVAL. */
brr_status brr_schedule_kmax(uint32_t kcap, brr_schedule *out);

/* Fills *out with the division-based comparison shuffle of the paper's
 * experiments (Sec. 7, Appendix A): one die per batch above 2^32 elements
 * (never reached: n < 2^32 here), then batches of two dice in the division
 * form while more than one element remains; no tail (a last batch at two
 * elements keeps one die). BRR_EINVAL for a null out. */
brr_status brr_schedule_naive2(brr_schedule *out);

/* Number of batches (= words on first attempts) of an n-element shuffle that
 * performs `steps` Fisher-Yates steps (steps = n - 1 for a full shuffle).
 * Returns 0 for an invalid schedule. */
uint64_t brr_schedule_batches(const brr_schedule *sched, uint64_t n, uint64_t steps);

/* Checks a schedule for an n-element shuffle: every batch's bound product at
 * most 2^L (L = 32 for BRR_WORDS_PHILOX32, else 64), every non-zero upper
 * bound at least the product it guards, no element left unshuffled, a known
 * word stream (division steps need 64-bit words), reserved = 0. BRR_OK,
 * BRR_EINVAL or BRR_EOVERFLOW. */
brr_status brr_schedule_check(const brr_schedule *sched, uint64_t n);

/* Checks a schedule for every shuffle of at most max_n elements and every
 * sample from one (what a plan or a server may meet): the checks of
 * brr_schedule_check at max_n, and for every step the largest batch it can
 * roll at any such size, which is its first batch at size
 * min(max_n, n_above of the step before) (the tail's at min(max_n, the last
 * n_above)): its product at most 2^L and at most the step's non-zero upper
 * bound. brr_schedule_check(max_n) alone does not imply this, since where a
 * step's first batch falls depends on n; and, without a tail, a last step
 * that runs down to one element (n_above <= 1, else a shuffle of n_above
 * elements would roll nothing). BRR_OK, BRR_EINVAL or BRR_EOVERFLOW. */
brr_status brr_schedule_check_upto(const brr_schedule *sched, uint64_t max_n);

/* ------------------------------------------------------------------------ */
/* Planning: the cost model of Sec. 6.1 and schedules derived from it        */
/* ------------------------------------------------------------------------ */

/* Expected cost per die of a batch of k dice at size n with L-bit words
 * (Sec. 6.1): ((c_rng + k) / (1 - p2) + (c_div + k - 1) * p1) / k with
 * p1 = n^(falling k) / 2^L and p2 = (2^L mod n^(falling k)) / 2^L, in units
 * of one multiplication. +inf when n^(falling k) > 2^L; NaN for k = 0 or
 * L outside 1..64. */
double brr_cost_per_die(uint64_t n, uint32_t k, uint32_t L, double c_rng, double c_div);

/* n_k for k = 2..kmax (Table 2): the largest n such that a batch of k costs
 * less per die than a batch of k - 1 at every size from k up to n.
 * out_nk: host u64[kmax + 1], entries 0 and 1 set to 0. With L = 64,
 * c_rng = 2, c_div = 16 this is the paper's table. 8 <= L <= 64,
 * 2 <= kmax <= BRR_MAX_K. */
brr_status brr_cost_thresholds(uint32_t L, uint32_t kmax, double c_rng, double c_div,
                               uint64_t *out_nk);

/* A schedule from the cost model (64-bit words unless BRR_COSTS_L32): one
 * die above n_2, then k
 * dice while more than n_{k+1} elements remain (k up to kmax), guards
 * u_k = n_k^k, and a last batch of at most kmax - 1 dice. Flags:
 * BRR_COSTS_POW2 rounds each n_k down to a power of two first, as the paper
 * does for its experiments (Sec. 6.1) -- kmax = 6, c_rng = 2, c_div = 16 with
 * this flag gives shuffle_6 exactly; BRR_COSTS_SMOOTH replaces p2 by its mean
 * p1 / 2, which makes n_k a bisection (microseconds) instead of the exact
 * first-crossing scan of brr_cost_thresholds (seconds for k = 2). */
#define BRR_COSTS_POW2 1
#define BRR_COSTS_SMOOTH 2
#define BRR_COSTS_L32 4 /* the cost model at L = 32; the schedule reads BRR_WORDS_PHILOX32 */
brr_status brr_schedule_from_costs(uint32_t kmax, double c_rng, double c_div, int flags,
                                   brr_schedule *out);

/* ------------------------------------------------------------------------ */
/* Dice streams (Theorem 1; Algorithm 3 per group, Algorithm 2 for a constant) */
/* ------------------------------------------------------------------------ */

/* out[j] is uniform in [0, bounds[j]), j < count. Bounds are grouped k at a
 * time (group s = bounds[s*k .. s*k+k-1]; the last group keeps count mod k
 * bounds when non-zero) and each group is rolled from one word, b_1 applied
 * first (a_1 most significant digit). 1 <= k <= 8.
 * d_bounds: u32[count], read only. d_out: u32[count], written; must not
 * overlap d_bounds. A zero bound or a group product above 2^64 is reported
 * by brr_sync_status (BRR_EINVAL / BRR_EOVERFLOW). */
brr_status brr_dice(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                    uint64_t seed, uint64_t inst, void *stream);

/* Sampling with replacement: out[j] uniform in [0, bound), k dice per word,
 * the threshold 2^64 mod bound^k computed once (Algorithm 2). Produces
 * exactly what brr_dice produces for a constant bounds array. bound >= 1,
 * 1 <= k <= 8, bound^k <= 2^64 (else BRR_EOVERFLOW). */
brr_status brr_dice_const(uint32_t bound, uint32_t *d_out, uint64_t count, uint32_t k,
                          uint64_t seed, uint64_t inst, void *stream);

/* Algorithm 2 for any tuple of bounds known ahead of time (the
 * known-threshold case of Sec. 5): group g rolls h_bounds[0..k) from one
 * word, out[g*k + i] uniform in [0, h_bounds[i]); the threshold 2^64 mod
 * (b_1 ... b_k) is computed once on the host (and once more for a short last
 * group, which holds the first count mod k bounds of the tuple). Produces
 * exactly what brr_dice produces for the tuple repeated over count bounds.
 * h_bounds: host u32[k], read during the call; 1 <= k <= 8; a zero bound is
 * BRR_EINVAL, a product above 2^64 BRR_EOVERFLOW. */
brr_status brr_dice_tuple(const uint32_t *h_bounds, uint32_t k, uint32_t *d_out, uint64_t count,
                          uint64_t seed, uint64_t inst, void *stream);

/* The division-based form of batched dice (Sec. 2.1, the comparison that the
 * paper's method replaces): each group rolls one value V uniform in
 * [0, b_1 ... b_k) by Lemire's method (Sec. 2) on the same words as brr_dice
 * (attempt a of group s reads word a*S + s; the acceptance test is the same,
 * so both forms read the same words), then takes its dice as successive
 * remainders of quotients: a_1 = V mod b_1, V <- V div b_1, a_2 = V mod b_2,
 * and so on (k - 1 integer divisions per group). Per group, brr_dice and
 * this form write the same V in mixed radix, most and least significant
 * digit first respectively. Arguments, grouping and errors as brr_dice. */
brr_status brr_dice_div(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                        uint64_t seed, uint64_t inst, void *stream);

/* The dice stream of brr_dice with a second word source: ChaCha20
 * (Bernstein 2008) in counter mode, the slow cryptographic generator of the
 * paper's experiments (Sec. 7). Word c of instance `inst` under `seed` is
 * output words 2m, 2m+1 (low half first, m = c mod 8) of ChaCha20 block c/8,
 * whose input state holds the four constant words, key words
 * (lo32 seed, hi32 seed, 0, 0, 0, 0, 0, 0), the 64-bit block counter c/8 in
 * words 12-13 and the 64-bit nonce inst in words 14-15. Dice, acceptance,
 * attempt addressing (attempt a of group s reads word a*S + s), arguments
 * and errors as brr_dice. Groups rejected on their first word are rerolled
 * by a second kernel of persistent wavefronts from per-tile records in
 * device scratch (68 bytes per tile of 512 groups, plus up to 12 to align
 * the offsets to 16 bytes; up to 32 rejected groups a tile; the stream's
 * scratch buffer, see brr_release_scratch); a tile
 * with more, or every tile if the scratch cannot be had, rerolls in place
 * (the same dice, more slowly). */
brr_status brr_dice_chacha(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                           uint64_t seed, uint64_t inst, void *stream);

/* The dice stream of brr_dice at word width L = 32 (Theorem 1 holds for any
 * L, Sec. 4): each group is rolled from one 32-bit word with one 32x32 ->
 * 64-bit multiply per die, and accepted when the leftover is at least
 * 2^32 mod P (Algorithm 3). Word c of the 32-bit stream is the 32-bit half
 * c mod 2, low half first, of 64-bit word c/2 (so four dice groups share one
 * Philox block); attempt a of group s reads word a*S + s. The bound product
 * of a group must not exceed 2^32 (else BRR_EOVERFLOW through
 * brr_sync_status). Arguments, grouping and errors as brr_dice. */
brr_status brr_dice32(const uint32_t *d_bounds, uint32_t *d_out, uint64_t count, uint32_t k,
                      uint64_t seed, uint64_t inst, void *stream);

/* ------------------------------------------------------------------------ */
/* Shuffles (Algorithm 1 driven by Algorithm 4 batches)                     */
/* ------------------------------------------------------------------------ */

/* Shuffles d_data[0..n-1] in place. elem_bytes is 4 or 8. sched = NULL uses
 * shuffle_6. The result is the permutation that the sequential batched
 * Fisher-Yates shuffle produces: batch at size i rolls bounds i, i-1, ...,
 * i-k+1 and swaps z[i-1] with z[a_1] first. n <= 1 is a no-op;
 * n < 2^32. n above 16,384 takes device scratch of about 33 bytes plus
 * elem_bytes per element (brr_scratch_bytes) from the stream's scratch
 * buffer (see brr_release_scratch); BRR_ENOMEM if it cannot be had. */
brr_status brr_shuffle(void *d_data, uint64_t n, uint32_t elem_bytes, const brr_schedule *sched,
                       uint64_t seed, uint64_t inst, void *stream);

/* brr_shuffle for callers that cannot allocate (code under hip graph
 * capture, serving loops, harnesses that forbid allocation): the same
 * result as brr_shuffle with the same arguments, but nothing is allocated.
 * Arrays above 16,384 elements use a scratch array that the library holds
 * in device memory, one of BRR_NOALLOC_SCRATCH_BYTES per device, from the
 * first call on that device until the process ends. n is limited to
 * BRR_NOALLOC_MAX_N (2^21) elements; a larger n returns BRR_EINVAL with
 * nothing enqueued. Every call initialises the parts of the scratch it
 * reads, so no clearing is needed between calls. All calls on one device
 * share that one array: calls that may overlap on the device (on different
 * streams, or from several host threads without ordering) race and give
 * unspecified results; order them on one stream. Other arguments, results
 * and errors as brr_shuffle. */
#define BRR_NOALLOC_MAX_N (1ull << 21)
#define BRR_NOALLOC_SCRATCH_BYTES (96ull << 20)
brr_status brr_shuffle_noalloc(void *d_data, uint64_t n, uint32_t elem_bytes,
                               const brr_schedule *sched, uint64_t seed, uint64_t inst,
                               void *stream);

/* A plan for a batch of shuffles given in CSR form: shuffle q covers
 * elements offsets[q] .. offsets[q+1]-1 of one array and uses instance
 * inst_base + q. The plan sorts the shuffles into size classes (one lane,
 * one wavefront, one workgroup, or device-wide per shuffle), owns the device
 * copies of that classification, any scratch it needs, and a hip graph of
 * the launch sequence. h_offsets: host u64[count + 1], non-decreasing,
 * offsets[0] = 0. sched = NULL uses shuffle_6; it is copied. The graph is
 * captured once, on the plan's first run, and replayed by every later run:
 * its kernels read the run's data pointer, offsets pointer, seed and
 * instance from a small device block of the plan, which a kernel enqueued on
 * the caller's stream just before each replay writes. So a run with other
 * buffers, seed or instance needs no recapture and no host wait.
 * brr_plan_destroy waits for the plan's last run, then releases everything
 * the plan owns. */
typedef struct brr_plan brr_plan;
brr_status brr_plan_create(brr_plan **out, const uint64_t *h_offsets, uint64_t count,
                           uint32_t elem_bytes, const brr_schedule *sched);
void brr_plan_destroy(brr_plan *plan);

/* How many times the plan has captured its launch graph: 0 before its first
 * run with use_graph = 1 (and always 0 for a plan launched as a single
 * kernel, see brr_mapping), then 1 (the capture is never repeated). */
uint32_t brr_plan_captures(const brr_plan *plan);

/* Plan knobs for the size-class mapping; brr_plan_create uses defaults that
 * brr_plan_set_mapping may replace before the first run. lane_max: shuffles
 * with n <= lane_max run one per lane, the sequential batched Fisher-Yates
 * of Algorithm 4 on a byte permutation in LDS (at most 256; 0 = no lane
 * tier);
 * wave_max: n <= wave_max one per wavefront (at most 512); larger shuffles
 * one per workgroup with their index arrays in LDS, in classes of 256, 256,
 * 512 and 1024 threads up to 2048, 4096, 8192 and 16384 elements, using
 * classes up to wg_threads (256, 512 or 1024) threads; larger ones one per
 * workgroup in peels of whole batches (up to 2^20 elements), else
 * device-wide with device scratch. use_graph: 1 = capture the launch sequence once
 * and replay it as a hip graph (a plan whose arrays all fall in one class
 * other than the device-wide one is a single kernel, which it launches
 * directly either way: one kernel launch costs less than a graph launch).
 * Every mapping gives the same output; an out-of-range knob, or a call
 * after the first run, is BRR_EINVAL. */
typedef struct {
    uint32_t lane_max;
    uint32_t wave_max;
    uint32_t wg_threads;
    uint32_t use_graph;
} brr_mapping;
brr_status brr_plan_get_mapping(const brr_plan *plan, brr_mapping *out);
brr_status brr_plan_set_mapping(brr_plan *plan, const brr_mapping *m);

/* Shuffles every array of the batch in place, as brr_shuffle would with
 * inst = inst_base + q. d_offsets: device copy of the plan's offsets (the
 * plan checks nothing on the device side; they must match). plan = NULL
 * builds a temporary plan from a synchronous copy of d_offsets. */
brr_status brr_shuffle_batched(void *d_data, const uint64_t *d_offsets, uint64_t count,
                               uint32_t elem_bytes, brr_plan *plan, uint64_t seed,
                               uint64_t inst_base, void *stream);

/* ------------------------------------------------------------------------ */
/* Autotuning (batch sizes are hardware-dependent, Sec. 6.1)                */
/* ------------------------------------------------------------------------ */

/* Times brr_dice for every k = 1..8 with max_bound^k <= 2^64 on a synthetic
 * stream of min(count, 2^26) bounds uniform in [1, max_bound] (device
 * scratch from the stream-ordered allocator), and returns the fastest k.
 * ms_per_k: host float[9] or NULL; entry k gets the time of one stream
 * (0 for k not tried). Results are cached per (bit length of max_bound,
 * count rounded to a power of two). Synchronizes `stream`. */
brr_status brr_dice_autotune(uint32_t max_bound, uint64_t count, void *stream, uint32_t *best_k,
                             float *ms_per_k);

typedef struct {
    uint32_t candidates; /* configurations timed */
    float ms_best;       /* time of one batch under the chosen configuration */
    float ms_default;    /* time under the plan's configuration before tuning */
    brr_schedule schedule;
    brr_mapping mapping;
} brr_tune_report;

/* Chooses the plan's schedule and size-class mapping by timing candidates on
 * a device copy of the batch (the caller's data is not modified): the plan's
 * own configuration, the paper's schedules and schedules derived from the
 * cost model (brr_schedule_from_costs) for several maximum batch sizes and
 * generator/division cost ratios, under wavefront-tier limits of 64..512.
 * Every candidate is exactly uniform (Theorem 1 holds for any schedule), so
 * the choice changes only speed and the word stream consumed. The plan then
 * uses the chosen configuration (brr_plan_get_schedule / get_mapping report
 * it). Each candidate's time is the median of five single runs after one
 * untimed run (report->ms_*). Must precede the plan's first run;
 * synchronizes `stream`. report may be NULL. */
brr_status brr_plan_autotune(brr_plan *plan, const void *d_data, const uint64_t *d_offsets,
                             uint64_t seed, uint64_t inst_base, void *stream,
                             brr_tune_report *report);

/* The schedule a plan uses (its creation argument, or the autotuner's choice). */
brr_status brr_plan_get_schedule(const brr_plan *plan, brr_schedule *out);

/* ------------------------------------------------------------------------ */
/* Learned plan-cost model                                                  */
/* ------------------------------------------------------------------------ */

/* A small multilayer perceptron, y = W3' tanh(W2' tanh(W1' x + b1) + b2) + b3
 * (n_in inputs, two hidden layers of `hidden`, one output, FP32, device
 * resident), trained by mean squared error with Adam in the library's own
 * kernels. It predicts the log-time of a batch under a candidate plan from
 * brr_plan_features; the autotuner uses it to rank candidates. It never
 * touches random words, rolls or swaps, so outputs stay exactly uniform.
 * Parameters are laid out W1[n_in][hidden], b1, W2[hidden][hidden], b2,
 * W3[hidden], b3, row-major, as float. Weights start Glorot-uniform from
 * `seed`, biases zero. Device pointers d_*: float, row-major [batch][n_in]
 * inputs, [batch] outputs/targets. */
typedef struct brr_mlp brr_mlp;
brr_status brr_mlp_create(brr_mlp **out, uint32_t n_in, uint32_t hidden, uint64_t seed);
void brr_mlp_destroy(brr_mlp *net);
uint64_t brr_mlp_num_params(const brr_mlp *net);
brr_status brr_mlp_get_params(const brr_mlp *net, float *h_out); /* synchronous */
brr_status brr_mlp_set_params(brr_mlp *net, const float *h_in);  /* synchronous */
brr_status brr_mlp_get_grads(const brr_mlp *net, float *h_out);  /* synchronous */
brr_status brr_mlp_forward(brr_mlp *net, const float *d_x, uint32_t batch, float *d_y,
                           void *stream);
/* Gradients of mean((y - t)^2) over the batch into the net's gradient
 * buffer; the loss into *d_loss (device float, may be NULL). */
brr_status brr_mlp_backward(brr_mlp *net, const float *d_x, const float *d_t, uint32_t batch,
                            float *d_loss, void *stream);
brr_status brr_mlp_adam_step(brr_mlp *net, float lr, void *stream);
/* steps x (backward + Adam) on one batch; final loss to *h_final_loss.
 * Synchronizes `stream`. */
brr_status brr_mlp_train(brr_mlp *net, const float *d_x, const float *d_t, uint32_t batch,
                         uint32_t steps, float lr, float *h_final_loss, void *stream);

#define BRR_PLAN_FEATURES 16
/* Features of a batch (CSR host offsets) under a schedule and wavefront-tier
 * limit: log total size, log count, payload width, element fractions by
 * size band, mean and spread of log2 n, words per step, fractions of dice
 * in batches of >= 4 and <= 2, largest batch, log wavefront limit, element
 * fraction in the wavefront tier. out: host float[BRR_PLAN_FEATURES]. */
brr_status brr_plan_features(const uint64_t *h_offsets, uint64_t count, uint32_t elem_bytes,
                             const brr_schedule *sched, uint32_t wave_max, float *out);

/* brr_plan_autotune guided by a trained model: every candidate is ranked by
 * predicted time and only the plan's own configuration and the `top` best
 * predicted ones are timed. */
brr_status brr_plan_autotune_learned(brr_plan *plan, brr_mlp *model, uint32_t top,
                                     const void *d_data, const uint64_t *d_offsets, uint64_t seed,
                                     uint64_t inst_base, void *stream, brr_tune_report *report);

/* ------------------------------------------------------------------------ */
/* Sampling without replacement (partial Fisher-Yates, Algorithm 4 Ensure)  */
/* ------------------------------------------------------------------------ */

/* Sampling without replacement (Algorithm 4's partial shuffle, Sec. 6):
 * d_out[t] = z[n-1-t], t < m, where z is d_data after the first m steps of
 * the scheduled shuffle of d_data (the last batch cut to the dice needed).
 * d_data is not modified. m <= n, elem_bytes 4 or 8, n < 2^32. Above 16,384
 * elements the work and the device scratch are O(m), whatever n: only the
 * m steps are rolled and resolved, and only the at most 2m positions they
 * touch are read (brr_scratch_bytes gives the scratch; it comes from the
 * stream's scratch buffer, see brr_release_scratch). */
brr_status brr_sample(const void *d_data, uint64_t n, uint64_t m, uint32_t elem_bytes, void *d_out,
                      const brr_schedule *sched, uint64_t seed, uint64_t inst, void *stream);

/* Bytes of device scratch that brr_shuffle (m = 0) or brr_sample (m > 0)
 * takes for an array of n elements of elem_bytes each: 0 up to 16,384
 * elements (one workgroup's LDS does), else about 33 + elem_bytes bytes per
 * element for a shuffle and 28 bytes per sampled element for a sample.
 * Returns 0 for invalid sizes (elem_bytes not 4 or 8, m > n, n >= 2^32). */
uint64_t brr_scratch_bytes(uint64_t n, uint64_t m, uint32_t elem_bytes);

/* Scratch of brr_shuffle, brr_sample, brr_dice_chacha and the server's
 * large requests: the library keeps one device buffer per (device, stream),
 * allocated with hipMalloc the first time a call on that stream needs
 * scratch and replaced by a larger one (after the stream's earlier work has
 * ended) when a later call needs more; calls on one stream share it in
 * stream order, so those calls stay asynchronous. A server frees its
 * streams' buffers when it is destroyed; the others are held until this
 * call, which waits for each device that holds one to finish its work and
 * frees them all (later calls allocate again). Not to be called while calls
 * that use the buffers are being made from other threads. BRR_EHIP if a
 * wait or a free fails. */
brr_status brr_release_scratch(void);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of shuffle and sample requests              */
/* ------------------------------------------------------------------------ */

/* A server admits requests in arrival order as in-flight slots and its
 * device-scratch budget allow, and retires them when their completion
 * events fire (continuous batching). What one pass of its worker admits is
 * launched together: requests of at most 16,384 elements as one launch per
 * size class and element width (one workgroup each), larger ones each on
 * one of a pool of HIP streams, all overlapping on the device. Each
 * session's generator counter lives on the device: request j of session s
 * (j = 0, 1, ... in submission order) uses instance s * 2^40 + j, claimed by
 * a kernel in submission order, so a result depends only on (seed, session,
 * j, inputs), never on the mix it ran in or on what ran beside it. Requests
 * run concurrently and may finish in any order, also within a session: a
 * buffer must not be used by two requests in flight at once. A request that
 * needs more scratch than the whole budget still runs, alone. Shuffles
 * follow brr_shuffle, samples brr_sample, with the server's schedule; a
 * large request uses the scratch buffer of its stream (brr_release_scratch),
 * so the device memory held is up to nstreams times the largest request's
 * scratch, whatever the budget admits at once. */
typedef struct brr_server brr_server;

typedef struct {
    uint64_t hbm_budget;        /* bytes of device scratch in use at once */
    uint32_t max_inflight;      /* requests on the device at once */
    uint32_t nstreams;          /* HIP streams (1..64) */
    uint64_t seed;              /* word-stream seed of every request */
    const brr_schedule *schedule; /* NULL = shuffle_6; copied */
} brr_server_config;

#define BRR_REQ_SHUFFLE 1u
#define BRR_REQ_SAMPLE 2u

typedef struct {
    uint32_t kind;       /* BRR_REQ_SHUFFLE (in place) or BRR_REQ_SAMPLE */
    uint32_t elem_bytes; /* 4 or 8 */
    uint64_t session;    /* < 2^24; names the counter and the stream */
    void *d_data;        /* device, n elements; must stay valid until completion */
    uint64_t n;
    uint64_t m;          /* sample size (samples only), m <= n */
    void *d_out;         /* device, m elements (samples only) */
} brr_request;

typedef struct {
    uint64_t completed, elements; /* requests and elements (shuffled or sampled) */
    double p50_us, p99_us, mean_us, max_us; /* latency, submission to completion */
    double wall_s, requests_per_s, elements_per_s; /* first submission to last completion */
    uint32_t peak_inflight;
    uint64_t peak_footprint;      /* bytes of scratch admitted at once */
} brr_server_stats;

brr_status brr_server_create(brr_server **out, const brr_server_config *cfg);
/* Queues a request; *id names it for brr_server_wait. */
brr_status brr_server_submit(brr_server *server, const brr_request *req, uint64_t *id);
/* Waits for one request (BRR_EDEVICE on time-out); its latency in
 * *latency_us (may be NULL). The id is released. */
brr_status brr_server_wait(brr_server *server, uint64_t id, double timeout_s, double *latency_us);
/* Waits until nothing is pending or in flight, releasing finished ids. */
brr_status brr_server_drain(brr_server *server, double timeout_s);
brr_status brr_server_get_stats(brr_server *server, brr_server_stats *out);
brr_status brr_server_reset_stats(brr_server *server);
/* The device counter of a session (requests claimed so far); synchronizes
 * the server's claims. */
brr_status brr_server_session_counter(brr_server *server, uint64_t session, uint64_t *value);
/* Finishes every queued request, then releases the server. */
void brr_server_destroy(brr_server *server);

/* ------------------------------------------------------------------------ */
/* Status                                                                   */
/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */

/* Measures how many dice per second the device's vector ALUs can chain: one
 * Theorem 1 step (two 32x32+64 -> 64-bit multiply-adds, Sec. 4) per die, in
 * independent chains on every compute unit, `iters` steps per chain, with no
 * memory traffic and no word generation. It is the VALU ceiling of a dice
 * stream, for the roofline. Runs two launches on the null stream and
 * synchronizes it; *dice_per_s receives the rate of the second. */
brr_status brr_probe_chain_rate(uint32_t iters, double *dice_per_s);

/* Measures the memory ceiling of a stream that reads and writes the same
 * number of bytes, as a dice stream does: copies `bytes` (a multiple of 16)
 * from device buffer src to device buffer dst (both 16-byte aligned, not
 * overlapping, owned by the caller) with the fastest copy shape measured on
 * MI355X (one 16-byte nontemporal load and store per lane, one contiguous
 * tile per workgroup), once to warm up and then `reps` times on `stream`,
 * which it synchronizes. *bytes_per_s receives
 * the bytes moved (read plus written, 2 * bytes per copy) per second over
 * the timed copies. BRR_EINVAL for null pointers, zero sizes, misaligned
 * pointers or sizes. */
brr_status brr_probe_copy_rate(const void *src, void *dst, uint64_t bytes, uint32_t reps,
                               void *stream, double *bytes_per_s);

/* ------------------------------------------------------------------------ */

/* Waits for `stream`, then returns and clears the first device-detected
 * error of the current device (BRR_OK if none). */
brr_status brr_sync_status(void *stream);

/* Static description of a status code. */
const char *brr_strerror(brr_status status);

#ifdef __cplusplus
}
#endif

#endif /* BRR_H */
