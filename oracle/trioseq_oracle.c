/*
 * CPU oracle for exact 3-way alignment scoring (global, semi-global and local).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the library or its Python binding
 * links, loads or calls this file; only the test-suite, the smoke check and
 * the CPU baseline of the benchmark do. It shares no code, header or table
 * with the GPU path.
 *
 * What it computes (paper, Section II, Eq. 1 and the "Global Alignments"
 * initialisation): for sequences S0, S1, S2 of lengths a, b, c,
 *
 *   M[i][j][k] = max over the seven moves that decrement a non-empty subset
 *                of {i, j, k}, of  M[predecessor] + SOP(column of the move),
 *
 * where the column holds S0[i-1] if i is decremented, else a gap (and the same
 * for j with S1, k with S2). SOP(x, y, z) = s(x,y) + s(x,z) + s(y,z), with
 * s(r, r') = sub[r][r'] for two residues, s(r, -) = s(-, r) = gap for a residue
 * and a gap, and s(-, -) = 0. M[0][0][0] = 0 and the global score is M[a][b][c].
 *
 * Readings (the paper's text leaves these open):
 *  - "v = -infinity" for the global variant is taken as: a move whose
 *    predecessor index would be negative does not exist. With that rule the
 *    recurrence itself produces the printed axis values M[i][0][0] = 2*i*gap
 *    and the three face recurrences, so no separate initialisation code exists.
 *  - gap is the score of one residue-versus-gap pair (normally negative); the
 *    axis value 2*i*gap is what a column of one residue and two gaps scores.
 *  - The first face recurrence prints its third term as M[i][j][0] (itself);
 *    it is read as M[i][j-1][0] by symmetry with the other two faces. The
 *    "no negative index" rule above gives exactly that reading.
 *
 * Arithmetic is int64, so no intermediate can overflow for any input the
 * library accepts. Memory is two (b+1) x (c+1) slices of int64.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NEG_INF INT64_MIN

static int64_t pair(const int32_t *sub, int x, int y) { return (int64_t)sub[4 * x + y]; }

/* Score of one triplet. Residues are codes 0..3. Returns 0 on success. */
int oracle_score(const uint8_t *s0, int64_t a, const uint8_t *s1, int64_t b,
                 const uint8_t *s2, int64_t c, const int32_t *sub, int32_t gap,
                 int64_t *out)
{
    const int64_t row = c + 1;
    const int64_t plane = (b + 1) * row;
    int64_t *prev = (int64_t *)malloc((size_t)plane * sizeof(int64_t));
    int64_t *cur = (int64_t *)malloc((size_t)plane * sizeof(int64_t));
    if (!prev || !cur) {
        free(prev);
        free(cur);
        return -1;
    }
    const int64_t g = gap;
    for (int64_t i = 0; i <= a; i++) {
        for (int64_t j = 0; j <= b; j++) {
            for (int64_t k = 0; k <= c; k++) {
                if (i == 0 && j == 0 && k == 0) {
                    cur[0] = 0;
                    continue;
                }
                int64_t best = NEG_INF, v;
                /* Column (S0[i-1], S1[j-1], S2[k-1]). */
                if (i > 0 && j > 0 && k > 0) {
                    int x = s0[i - 1], y = s1[j - 1], z = s2[k - 1];
                    v = prev[(j - 1) * row + (k - 1)] + pair(sub, x, y) + pair(sub, x, z) + pair(sub, y, z);
                    if (v > best) best = v;
                }
                /* Column (S0[i-1], S1[j-1], -): s(x,y) + s(x,-) + s(y,-). */
                if (i > 0 && j > 0) {
                    v = prev[(j - 1) * row + k] + pair(sub, s0[i - 1], s1[j - 1]) + g + g;
                    if (v > best) best = v;
                }
                /* Column (S0[i-1], -, S2[k-1]). */
                if (i > 0 && k > 0) {
                    v = prev[j * row + (k - 1)] + pair(sub, s0[i - 1], s2[k - 1]) + g + g;
                    if (v > best) best = v;
                }
                /* Column (-, S1[j-1], S2[k-1]). */
                if (j > 0 && k > 0) {
                    v = cur[(j - 1) * row + (k - 1)] + pair(sub, s1[j - 1], s2[k - 1]) + g + g;
                    if (v > best) best = v;
                }
                /* Columns with one residue and two gaps: s(r,-) + s(r,-) + s(-,-). */
                if (i > 0) {
                    v = prev[j * row + k] + g + g;
                    if (v > best) best = v;
                }
                if (j > 0) {
                    v = cur[(j - 1) * row + k] + g + g;
                    if (v > best) best = v;
                }
                if (k > 0) {
                    v = cur[j * row + (k - 1)] + g + g;
                    if (v > best) best = v;
                }
                cur[j * row + k] = best;
            }
        }
        int64_t *t = prev;
        prev = cur;
        cur = t;
    }
    *out = prev[b * row + c];
    free(prev);
    free(cur);
    return 0;
}

/*
 * Semi-global variant (paper, Section II, "Semi-Global Alignments"): v stays
 * -infinity (a move with a negative predecessor index does not exist), the
 * three axes are set to 0 (M[i][0][0] = M[0][j][0] = M[0][0][k] = 0, whatever
 * the moves along them would give), every other cell follows Eq. 1, and the
 * score is the largest value on the last slices i = a, j = b or k = c.
 * Same int64 two-slice loop as oracle_score.
 */
int oracle_score_semiglobal(const uint8_t *s0, int64_t a, const uint8_t *s1, int64_t b,
                            const uint8_t *s2, int64_t c, const int32_t *sub, int32_t gap,
                            int64_t *out)
{
    const int64_t stride = c + 1;
    int64_t *older = (int64_t *)malloc((size_t)((b + 1) * stride) * sizeof(int64_t));
    int64_t *newer = (int64_t *)malloc((size_t)((b + 1) * stride) * sizeof(int64_t));
    if (!older || !newer) {
        free(older);
        free(newer);
        return -1;
    }
    const int64_t gg = 2 * (int64_t)gap; /* one residue and two gaps */
    int64_t answer = NEG_INF;
    for (int64_t i = 0; i <= a; i++) {
        for (int64_t j = 0; j <= b; j++) {
            for (int64_t k = 0; k <= c; k++) {
                int64_t m;
                if ((i == 0) + (j == 0) + (k == 0) >= 2) {
                    m = 0; /* an axis */
                } else {
                    const int x = i ? s0[i - 1] : 0, y = j ? s1[j - 1] : 0, z = k ? s2[k - 1] : 0;
                    m = NEG_INF;
                    int64_t t;
                    if (i && j && k) {
                        t = older[(j - 1) * stride + (k - 1)] + pair(sub, y, z) + pair(sub, x, y) + pair(sub, x, z);
                        if (t > m) m = t;
                    }
                    if (j && k) {
                        t = newer[(j - 1) * stride + (k - 1)] + gg + pair(sub, y, z);
                        if (t > m) m = t;
                    }
                    if (i && k) {
                        t = older[j * stride + (k - 1)] + gg + pair(sub, x, z);
                        if (t > m) m = t;
                    }
                    if (i && j) {
                        t = older[(j - 1) * stride + k] + gg + pair(sub, x, y);
                        if (t > m) m = t;
                    }
                    if (k) {
                        t = newer[j * stride + (k - 1)] + gg;
                        if (t > m) m = t;
                    }
                    if (j) {
                        t = newer[(j - 1) * stride + k] + gg;
                        if (t > m) m = t;
                    }
                    if (i) {
                        t = older[j * stride + k] + gg;
                        if (t > m) m = t;
                    }
                }
                newer[j * stride + k] = m;
                if ((i == a || j == b || k == c) && m > answer) answer = m;
            }
        }
        int64_t *sw = older;
        older = newer;
        newer = sw;
    }
    *out = answer;
    free(older);
    free(newer);
    return 0;
}

/*
 * Local variant (paper, Section II, "Local Alignments"): the initialisation of
 * the semi-global variant (M[i][0][0] = M[0][j][0] = M[0][0][k] = 0) with
 * v = 0 as an eighth candidate of Eq. 1 for every cell, so no value is
 * negative; an alignment may start and end anywhere, and the score is the
 * largest value anywhere in the tensor. With v = 0 in every cell the axis
 * values are max(0, moves) = 0 for a non-positive gap, which is the stated
 * initialisation; the recurrence below applies v = 0 to every cell, axes
 * included. Same int64 two-slice loop as oracle_score.
 */
int oracle_score_local(const uint8_t *s0, int64_t a, const uint8_t *s1, int64_t b,
                       const uint8_t *s2, int64_t c, const int32_t *sub, int32_t gap,
                       int64_t *out)
{
    const int64_t w = c + 1;
    int64_t *last = (int64_t *)malloc((size_t)((b + 1) * w) * sizeof(int64_t));
    int64_t *here = (int64_t *)malloc((size_t)((b + 1) * w) * sizeof(int64_t));
    if (!last || !here) {
        free(last);
        free(here);
        return -1;
    }
    const int64_t twogap = 2 * (int64_t)gap; /* a residue against two gaps */
    int64_t top = 0;
    for (int64_t i = 0; i <= a; i++) {
        for (int64_t j = 0; j <= b; j++) {
            for (int64_t k = 0; k <= c; k++) {
                const int x = i > 0 ? s0[i - 1] : 0, y = j > 0 ? s1[j - 1] : 0, z = k > 0 ? s2[k - 1] : 0;
                int64_t m = 0; /* v = 0: the eighth candidate */
                int64_t cand;
                if (i && j && k) {
                    cand = last[(j - 1) * w + k - 1] + (pair(sub, x, y) + pair(sub, x, z)) + pair(sub, y, z);
                    m = cand > m ? cand : m;
                }
                if (i && j) {
                    cand = last[(j - 1) * w + k] + pair(sub, x, y) + twogap;
                    m = cand > m ? cand : m;
                }
                if (i && k) {
                    cand = last[j * w + k - 1] + pair(sub, x, z) + twogap;
                    m = cand > m ? cand : m;
                }
                if (j && k) {
                    cand = here[(j - 1) * w + k - 1] + pair(sub, y, z) + twogap;
                    m = cand > m ? cand : m;
                }
                if (i) {
                    cand = last[j * w + k] + twogap;
                    m = cand > m ? cand : m;
                }
                if (j) {
                    cand = here[(j - 1) * w + k] + twogap;
                    m = cand > m ? cand : m;
                }
                if (k) {
                    cand = here[j * w + k - 1] + twogap;
                    m = cand > m ? cand : m;
                }
                here[j * w + k] = m;
                top = m > top ? m : top;
            }
        }
        int64_t *t = last;
        last = here;
        here = t;
    }
    *out = top;
    free(last);
    free(here);
    return 0;
}

/* Many triplets on a pool of plain threads, one triplet at a time each.
 * seqs holds all residues back to back; off[3*t+s] / len[3*t+s] locate
 * sequence s of triplet t. */
typedef struct {
    const uint8_t *seqs;
    const int64_t *off;
    const int64_t *len;
    int64_t n;
    const int32_t *sub;
    int32_t gap;
    int kind; /* 0 global, 2 local */
    int64_t *out;
    int64_t next;
    int failed;
    pthread_mutex_t lock;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *job = (batch_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        int64_t t = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (t >= job->n) return NULL;
        const int64_t *o = job->off + 3 * t, *l = job->len + 3 * t;
        int rc = job->kind == 2
                     ? oracle_score_local(job->seqs + o[0], l[0], job->seqs + o[1], l[1],
                                          job->seqs + o[2], l[2], job->sub, job->gap, job->out + t)
                 : job->kind == 1
                     ? oracle_score_semiglobal(job->seqs + o[0], l[0], job->seqs + o[1], l[1],
                                               job->seqs + o[2], l[2], job->sub, job->gap, job->out + t)
                     : oracle_score(job->seqs + o[0], l[0], job->seqs + o[1], l[1], job->seqs + o[2],
                                    l[2], job->sub, job->gap, job->out + t);
        if (rc != 0) {
            pthread_mutex_lock(&job->lock);
            job->failed = 1;
            pthread_mutex_unlock(&job->lock);
        }
    }
}

int oracle_score_batch(const uint8_t *seqs, const int64_t *off, const int64_t *len, int64_t n,
                       const int32_t *sub, int32_t gap, int64_t *out, int threads, int kind)
{
    batch_job job;
    memset(&job, 0, sizeof job);
    job.seqs = seqs;
    job.off = off;
    job.len = len;
    job.n = n;
    job.sub = sub;
    job.gap = gap;
    job.kind = kind;
    job.out = out;
    pthread_mutex_init(&job.lock, NULL);
    if (threads < 1) threads = 1;
    pthread_t *tid = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)threads);
    int started = 0;
    for (int w = 0; w < threads; w++)
        if (pthread_create(&tid[started], NULL, batch_worker, &job) == 0) started++;
    if (started == 0) batch_worker(&job);
    for (int w = 0; w < started; w++) pthread_join(tid[w], NULL);
    free(tid);
    pthread_mutex_destroy(&job.lock);
    return job.failed ? -1 : 0;
}
