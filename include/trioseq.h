/*
 * trioseq.h -- C ABI of libtrioseq: exact global 3-way (triplet) alignment
 * scoring of DNA on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Section II, Eq. 1, sum-of-pairs definition and the
 * "Global Alignments" initialisation): for sequences S0, S1, S2 of lengths
 * a, b, c, the optimal global sum-of-pairs score is M[a][b][c] of the tensor
 *   M[i][j][k] = max over the 7 moves that consume a non-empty subset of the
 *                next residues of S0, S1, S2, of  M[predecessor] + SOP(column),
 *   SOP(x,y,z) = s(x,y) + s(x,z) + s(y,z),  s(r,r') = sub[r][r'],
 *   s(r,-) = s(-,r) = gap,  s(-,-) = 0,  M[0][0][0] = 0,
 * which equals the best summed column score over all 3-row global alignments.
 * Scores are exact int32; there is no tolerance.
 *
 * Conventions for every call:
 *  - Residues are A, C, G, T (either case) with codes 0, 1, 2, 3. Anything
 *    else is rejected with TRIOSEQ_ERR_BAD_RESIDUE.
 *  - Packed form: 16 residues per uint32, residue p of a sequence at bits
 *    2*(p % 16) .. 2*(p % 16)+1 of word p / 16 (trioseq_pack).
 *  - Lengths may be 0. A triplet's cell count is a*b*c (the paper's TCUPS
 *    definition, Section V-A).
 *  - Every call returns a trioseq_status; on error the outputs are left
 *    untouched and trioseq_last_error() returns a message for the calling
 *    thread. Inputs are validated before any kernel is launched (a
 *    validation error launches nothing); batch validation is all-or-nothing
 *    and the message names the first bad triplet.
 *  - No C++ exception crosses this ABI.
 *  - "hip_stream" arguments take a hipStream_t (NULL = the null stream).
 */
#ifndef TRIOSEQ_H
#define TRIOSEQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum trioseq_status {
  TRIOSEQ_OK = 0,
  TRIOSEQ_ERR_INVALID_ARG = -1, /* null pointer, asymmetric matrix, bad option */
  TRIOSEQ_ERR_BAD_RESIDUE = -2, /* a character outside ACGTacgt */
  TRIOSEQ_ERR_TOO_LARGE = -3,   /* lengths beyond what the kernels support */
  TRIOSEQ_ERR_OVERFLOW = -4,    /* the score range could exceed int32 headroom */
  TRIOSEQ_ERR_NOMEM = -5,       /* host or device allocation failed */
  TRIOSEQ_ERR_DEVICE = -6,      /* a HIP call failed; message has the HIP error */
  TRIOSEQ_ERR_BUSY = -7,        /* server queue full; retry later */
  TRIOSEQ_ERR_TIMEOUT = -8,     /* wait ended before the result was ready */
  TRIOSEQ_ERR_CLOSED = -9       /* server is shutting down */
} trioseq_status;

/* Alignment kinds (Section II: the value v of Eq. 1 and the tensor's
 * initialisation select them).
 *  GLOBAL:      v = -infinity, M[0][0][0] = 0, axes M[i][0][0] = 2*i*gap (and
 *               likewise for j, k); the score is M[a][b][c].
 *  SEMI_GLOBAL: v = -infinity, the three axes are 0; the score is the best
 *               cell on the last slices (i = a, j = b or k = c).
 *  LOCAL:       the semi-global initialisation with v = 0 (no cell below 0);
 *               the score is the best cell of the tensor. */
typedef enum trioseq_kind {
  TRIOSEQ_GLOBAL = 0,
  TRIOSEQ_SEMI_GLOBAL = 1,
  TRIOSEQ_LOCAL = 2
} trioseq_kind;

/* Scoring scheme (Section II: sigma and the linear gap value alpha).
 * sub must be symmetric (the sum-of-pairs score treats the three sequences
 * alike). gap is the score of one residue against a gap (normally negative);
 * gap against gap always scores 0. Limits: every sub[x][y] - 2*gap lies in
 * [-127, 127] (the kernels keep these terms as bytes); SEMI_GLOBAL and LOCAL
 * need gap <= 0. kind is a trioseq_kind; semi-global and local plans support
 * 4 x 4 (the default) and 8 x 4 lane tiles at 2 waves per SIMD. */
typedef struct trioseq_scoring {
  int32_t sub[4][4];
  int32_t gap;
  int32_t kind;
} trioseq_scoring;

/* Fills sub with match on the diagonal and mismatch elsewhere; kind = GLOBAL. */
void trioseq_scoring_simple(trioseq_scoring* s, int32_t match, int32_t mismatch, int32_t gap);

/* One triplet as host ASCII. seq[s] may be NULL only if len[s] == 0. */
typedef struct trioseq_triplet {
  const char* seq[3];
  uint32_t len[3];
} trioseq_triplet;

/* Host helpers (no device work). */
/* Packs len ASCII residues into ceil(len/16) words (caller-owned). */
trioseq_status trioseq_pack(const char* seq, uint32_t len, uint32_t* words);
/* Default packed layout for n triplets: every sequence starts on a fresh
 * word, triplet-major. Writes 3n word offsets and the total word count. */
trioseq_status trioseq_packed_layout(const uint32_t* lens, size_t n, uint64_t* word_off,
                                     uint64_t* total_words);

/* Score of one triplet; synchronous. score is a host int32. */
trioseq_status trioseq_score(const trioseq_triplet* t, const trioseq_scoring* sc, int32_t* score);

/* Scores of n triplets, computed together (one persistent launch for the
 * batch; triplets that would hold the launch up are split over many
 * wavefronts). This is the paper's host pipeline (Section IV, Approach
 * Overview: triplets read on the host are sent to the GPU, the optimal
 * scores come back to the host), for a whole batch at once. t[0..n) are host
 * ASCII triplets; scores[0..n) is host memory owned by the caller. The call
 * keeps no pointer after it returns. Synchronous: returns when scores[0..n)
 * are written. Work is issued on hip_stream. The device workspace of the
 * last few batch shapes is cached per thread and reused when the same
 * lengths come again (no allocation on such calls). */
trioseq_status trioseq_score_batch(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc,
                                   int32_t* scores, void* hip_stream);

/* Scores of n triplets whose packed residues are already in device memory
 * (e.g. torch-owned buffers): the host pipeline of Section IV (Approach
 * Overview) with the sequences already uploaded. d_words: packed residues (trioseq_pack layout);
 * d_word_off / d_len: 3n entries each in device memory, sequence s of triplet
 * t starting at word d_word_off[3t+s] with d_len[3t+s] residues; d_scores: n
 * int32 in device memory. The offsets and lengths are read back first (the
 * call waits for hip_stream to reach it); the batch is then laid out, or the
 * layout of this thread's previous call is reused when lengths, offsets,
 * scoring and device are unchanged, and the scoring is enqueued on hip_stream
 * without waiting for it: d_words and d_scores must stay alive until the
 * stream passes this point. */
trioseq_status trioseq_score_batch_packed(const uint32_t* d_words, const uint64_t* d_word_off,
                                          const uint32_t* d_len, size_t n, const trioseq_scoring* sc,
                                          int32_t* d_scores, void* hip_stream);

/* trioseq_score_batch_packed for callers that cannot allocate device memory
 * (code under HIP graph capture of their own, tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, same scores, but the call
 * allocates and frees no device memory. Every device buffer it needs is
 * carved from a fixed scratch array of trioseq_noalloc_scratch_bytes()
 * (256 MiB) that the library holds on each GPU it runs on until the process
 * ends (its first call on a device looks the array up). Limits: the panel
 * faces of split triplets must fit 96 MiB (they take about a*b*c / 2 bytes:
 * a lone 512 x 512 x 512 triplet fits, the 1024 x 1000 x 1048 one does not)
 * and the rest of the batch's tables plus one wavefront's
 * workspace for its largest whole triplet must fit the remaining 160 MiB;
 * the call launches only as many wavefronts as that part holds workspaces
 * for, so large batches run on fewer wavefronts than
 * trioseq_score_batch_packed uses. Beyond these limits it returns
 * TRIOSEQ_ERR_TOO_LARGE and launches nothing. Every call on one GPU shares
 * that GPU's array and leaves its contents behind: calls that overlap in
 * time on one GPU (from two threads, or on two streams not ordered with each
 * other) race and may return wrong scores; callers must serialise them.
 * Synchronisation: reads the lengths and offsets back (waits for hip_stream
 * to reach the call), initialises on hip_stream and waits for that, then
 * enqueues the scoring without waiting. Not capturable itself. */
trioseq_status trioseq_score_batch_packed_noalloc(const uint32_t* d_words, const uint64_t* d_word_off,
                                                  const uint32_t* d_len, size_t n,
                                                  const trioseq_scoring* sc, int32_t* d_scores,
                                                  void* hip_stream);
/* Size of the scratch array behind trioseq_score_batch_packed_noalloc. */
uint64_t trioseq_noalloc_scratch_bytes(void);

/* Optimal global alignment of one triplet: the traceback (Section II, Eq. 1
 * for the scores; the alignment is recovered in linear space by Hirschberg's
 * divide and conquer, which the paper names for its traceback). row0, row1,
 * row2 (caller buffers of cap chars each) receive S0, S1, S2 as alignment
 * rows: residues in upper case, '-' for a gap, no terminating NUL; *ncols is
 * the number of columns and *score the sum-of-pairs score of the alignment,
 * which is the optimal global score. Requirements: sc->kind ==
 * TRIOSEQ_GLOBAL, every length <= 16384, cap >= len[0] + len[1] + len[2].
 * Synchronous; device work runs on hip_stream. On error nothing is written
 * to the outputs. */
trioseq_status trioseq_align(const trioseq_triplet* t, const trioseq_scoring* sc, char* row0,
                             char* row1, char* row2, uint32_t cap, uint32_t* ncols, int32_t* score,
                             void* hip_stream);

/* Optimal global alignments of n triplets, computed together (each level's
 * plane runs and all small sub-problems of the batch share launches). rows is
 * one caller buffer of 3 * sum_t cap_t chars, cap_t = len[0] + len[1] +
 * len[2] of triplet t; row s of triplet t occupies the cap_t chars at
 * rows + 3 * (cap_0 + ... + cap_{t-1}) + s * cap_t, its first ncols[t]
 * filled as in trioseq_align (no NULs). scores[t] is the optimal global
 * score. Requirements as trioseq_align. On error nothing is written. */
trioseq_status trioseq_align_batch(const trioseq_triplet* t, size_t n, const trioseq_scoring* sc,
                                   char* rows, uint32_t* ncols, int32_t* scores, void* hip_stream);

/* ---- Plans: device-resident batches (inputs already in HBM). ----------
 * The host side of Section IV's pipeline split in two: the layout of a batch
 * (which sequence is swept, which triplets are split into panel jobs, the
 * job order) is made once, and each run only launches the kernels. */

typedef struct trioseq_plan trioseq_plan;

typedef struct trioseq_plan_options {
  int32_t engine;         /* -1 auto (a lone triplet and very large ones are split
                             into panel jobs, the rest swept whole); 0 = every
                             triplet whole (one wavefront each); 1 = every triplet
                             split into panel jobs over many wavefronts */
  int32_t tile_rows;      /* lane tile rows; 0 = default (4) */
  int32_t tile_cols;      /* lane tile columns; 0 = default (4) */
  int32_t grid;           /* wavefronts to launch; 0 = fill the device */
  int32_t use_graph;      /* 1 = capture the launch sequence in a hipGraph and replay it */
  int32_t waves_per_simd; /* register budget of the kernel: 4 or 2; 0 = default */
  int32_t panel_group;    /* plans of panel jobs only: 1 = one panel per job, swept by
                             a workgroup of one computing and one staging wave; 4 =
                             strip jobs of four adjacent panels of one panel row,
                             swept by a workgroup of four such wave pairs that pass
                             the faces between the strip's panels in LDS (the
                             computing waves on distinct SIMDs); 0 = default */
  int32_t lane_exchange;  /* how the lanes of a wavefront pass tile edges to their
                             neighbours: 1 = through per-wave LDS slot arrays; 2 =
                             through ds_bpermute and DPP row shifts (no LDS round
                             trip); 0 = default */
  int32_t split_factor;   /* automatic engine: a triplet of a batch is split into panel
                             jobs when its cells exceed split_factor times the batch's
                             mean cells per wavefront (or 2.5e8); 0 = default (4) */
  int32_t half_split_min; /* automatic engine, one global or local triplet: scored by
                             two concurrent halves when its longest sequence has at
                             least this many residues; -1 = never; 0 = default (128,
                             and for local scoring only below 2048 residues) */
  int32_t packed;         /* 1 = int32 lanes; 2 = two triplets per lane, 16 bits each
                             (batches of whole triplets, any kind, whose substitution
                             terms sub - 2*gap are all >= 0 and whose values fit the
                             16-bit range; exact, like the int32 path; a batch that
                             does not qualify runs in int32); 0 = default (2 when the
                             lane tile is left to the library, else 1) */
  int32_t staging;        /* packed pairs: 1 = face rows staged through registers into
                             LDS; 2 = loaded straight into LDS (buffer loads to LDS);
                             0 = default */
} trioseq_plan_options;

typedef struct trioseq_plan_info {
  int32_t engine;         /* 0 all whole, 1 all split, 2 mixed */
  int32_t tile_rows, tile_cols, grid, waves_per_cu;
  int32_t panels;         /* panel jobs of split triplets */
  int32_t packed;         /* 1: two triplets per lane (16-bit halves); 0: int32 */
  uint64_t workspace_bytes;
  double cells;           /* sum of a*b*c over the batch */
} trioseq_plan_info;

/* Plans scores for n triplets whose lengths are lens[3t+s] (host array) and
 * whose packed words will live at word offsets word_off[3t+s] (host array;
 * NULL = trioseq_packed_layout). opts may be NULL. Allocates the device
 * workspace on the current HIP device; the plan owns it. */
trioseq_status trioseq_plan_create(const uint32_t* lens, const uint64_t* word_off, size_t n,
                                   const trioseq_scoring* sc, const trioseq_plan_options* opts,
                                   trioseq_plan** plan);
/* Enqueues the scoring of the planned batch on hip_stream. d_words: packed
 * residues in device memory; d_scores: n int32 in device memory (score of
 * triplet t at d_scores[t]). Asynchronous: both buffers must stay alive until
 * the stream passes this point. Runs of one plan must not overlap in time
 * (they share the plan's workspace). */
trioseq_status trioseq_plan_run(trioseq_plan* plan, const uint32_t* d_words, int32_t* d_scores,
                                void* hip_stream);
trioseq_status trioseq_plan_get_info(const trioseq_plan* plan, trioseq_plan_info* info);
trioseq_status trioseq_plan_destroy(trioseq_plan* plan);

/* ---- Autotuning. ------------------------------------------------------ */

typedef struct trioseq_tune_result {
  trioseq_plan_options best; /* options of the fastest accepted configuration */
  double best_ms;            /* its mean time per run */
  double reference_ms;       /* the reference configuration's (default options) */
  int32_t tried;             /* configurations timed */
  int32_t rejected;          /* configurations whose scores differed from the reference's */
} trioseq_tune_result;

/* Times candidate configurations on the caller's batch (lens, word_off and
 * d_words as for plans; reps timed runs each, on hip_stream) and returns the
 * fastest one whose scores equal the reference configuration's (the library
 * defaults), score for score (a candidate that differs is rejected and never
 * chosen). Candidates: every lane tile (panel shape) and register budget,
 * the register lane exchange, split factors 2, 8 and 16, strip workgroups,
 * and for one triplet half-split thresholds 128 and 512 and no half split.
 * The choice is remembered for the process, keyed by the batch's length
 * profile (triplet count, largest length and total cells, each bucketed by
 * powers of two): later plan_create calls that leave tile_rows, tile_cols and
 * waves_per_simd at 0 take all of its options that they leave at 0.
 * Synchronous. */
trioseq_status trioseq_autotune(const uint32_t* lens, const uint64_t* word_off, size_t n,
                                const trioseq_scoring* sc, const uint32_t* d_words, int32_t reps,
                                void* hip_stream, trioseq_tune_result* out);

/* ---- Serving: continuous batching of a request stream. ----------------
 * Section IV's host pipeline (triplets in, optimal scores back to the host)
 * run as a service: requests are admitted by device footprint into rounds
 * while earlier rounds still run, and each score reaches the host as soon as
 * its own triplet is done. */

typedef struct trioseq_server trioseq_server;

typedef struct trioseq_serve_config {
  int32_t device;            /* HIP device ordinal */
  uint64_t max_device_bytes; /* admission budget for workspaces (0 = 1/4 of HBM) */
  uint32_t max_len;          /* longest accepted sequence */
  uint32_t max_queue;        /* pending requests before submit returns BUSY */
  uint32_t max_batch;        /* triplets per device round (0 = automatic) */
  uint32_t max_inflight;     /* rounds in flight at once, each with its own
                                device arena and stream (0 = 4; at most 16);
                                max_device_bytes is shared among them */
} trioseq_serve_config;

typedef struct trioseq_result {
  uint64_t id;
  int32_t score;
  int32_t status;         /* trioseq_status of this request */
  uint64_t t_submit_ns;   /* steady clock at submit */
  uint64_t t_done_ns;     /* steady clock when the score reached the host */
} trioseq_result;

typedef struct trioseq_serve_stats {
  uint64_t submitted, completed, failed, rounds;
  double cells;           /* sum of a*b*c over completed requests */
  double busy_s;          /* wall time with at least one round in flight */
  double p50_ns, p99_ns;  /* submit-to-result latency over completed requests */
  double gcups;           /* cells / busy_s / 1e9: throughput while work was in flight */
} trioseq_serve_stats;

trioseq_status trioseq_serve_create(const trioseq_serve_config* cfg, const trioseq_scoring* sc,
                                    trioseq_server** srv);
/* Copies the triplet; never blocks on the device. BUSY when the queue is full. */
trioseq_status trioseq_serve_submit(trioseq_server* srv, const trioseq_triplet* t, uint64_t* id);
/* Moves up to cap finished results into out; never blocks. */
trioseq_status trioseq_serve_poll(trioseq_server* srv, trioseq_result* out, size_t cap,
                                  size_t* n_out);
/* Blocks until request id finishes (or timeout_ns passes; <0 = forever). The
 * result is consumed: it will not be returned by poll. */
trioseq_status trioseq_serve_wait(trioseq_server* srv, uint64_t id, trioseq_result* out,
                                  int64_t timeout_ns);
/* Statistics since create (both names are the same call). */
trioseq_status trioseq_serve_stats_get(trioseq_server* srv, trioseq_serve_stats* st);
trioseq_status trioseq_serve_get_stats(trioseq_server* srv, trioseq_serve_stats* st);
/* Stops admission, finishes queued and in-flight work, frees everything. */
trioseq_status trioseq_serve_destroy(trioseq_server* srv);

/* Bound on every wait of a kernel for another wavefront (a split triplet's
 * panels wait for their neighbours' faces), for launches and hipGraph
 * captures made after the call; ns = 0 restores the default of 2 s. A wait
 * that reaches it gives up: the run goes on and every score it produces for
 * a split triplet is INT32_MIN (served requests fail with
 * TRIOSEQ_ERR_DEVICE), never a wrong value. For tests of that failure path. */
void trioseq_set_wait_limit(uint64_t ns);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* trioseq_last_error(void);

/* Library version string. */
const char* trioseq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TRIOSEQ_H */
