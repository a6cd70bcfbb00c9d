/*
 * Multi-threaded form of the CPU raster oracle -- TEST INFRASTRUCTURE (the
 * CPU baseline of the benchmark times it on every host core).
 *
 * The render stage's result is, per pixel, the minimum key over the points
 * landing there (NARVis Sec. 3.2: the closest point wins the z-test; the key
 * packs fp32 depth bits above the point index).  A minimum does not depend
 * on the order or grouping of its operands, so T threads each render a
 * contiguous range of points into a private key buffer with the
 * single-threaded oracle's own routine, and the buffers are then merged by
 * an elementwise minimum: the merged buffer is the single-threaded result
 * bit for bit.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_EMPTY 0xFFFFFFFFFFFFFFFFull

void oracle_render_range(const float *x, const float *y, const float *z, uint64_t i0, uint64_t i1,
                         const float *M, float near_f, float far_f, int32_t W, int32_t H,
                         uint64_t *keys);

typedef struct {
    const float *x, *y, *z, *M;
    float near_f, far_f;
    int32_t W, H;
    uint64_t i0, i1;        /* render: this thread's points */
    int64_t p0, p1;         /* merge: this thread's pixels  */
    uint64_t *own;          /* this thread's key buffer     */
    uint64_t **all;         /* every thread's key buffer    */
    int nthreads;
    uint64_t *out;
} job;

static void *render_job(void *arg)
{
    job *j = (job *)arg;
    const int64_t npx = (int64_t)j->W * (int64_t)j->H;
    for (int64_t p = 0; p < npx; ++p) j->own[p] = ORACLE_EMPTY;
    oracle_render_range(j->x, j->y, j->z, j->i0, j->i1, j->M, j->near_f, j->far_f, j->W, j->H, j->own);
    return NULL;
}

static void *merge_job(void *arg)
{
    job *j = (job *)arg;
    for (int64_t p = j->p0; p < j->p1; ++p) {
        uint64_t k = ORACLE_EMPTY;
        for (int t = 0; t < j->nthreads; ++t)
            if (j->all[t][p] < k) k = j->all[t][p];
        j->out[p] = k;
    }
    return NULL;
}

/* keys[H*W] = the render stage over points [0, n) with `threads` threads.
 * Returns 0, or -1 when memory or threads could not be had. */
int oracle_render_mt(const float *x, const float *y, const float *z, uint64_t n,
                     const float *M, float near_f, float far_f, int32_t W, int32_t H,
                     uint64_t *keys, int threads)
{
    if (threads < 1) threads = 1;
    const int64_t npx = (int64_t)W * (int64_t)H;
    job *jobs = calloc((size_t)threads, sizeof(job));
    uint64_t **bufs = calloc((size_t)threads, sizeof(uint64_t *));
    pthread_t *tid = calloc((size_t)threads, sizeof(pthread_t));
    int ok = jobs && bufs && tid;
    for (int t = 0; ok && t < threads; ++t) {
        bufs[t] = malloc((size_t)npx * sizeof(uint64_t));
        ok = bufs[t] != NULL;
    }
    int started = 0;
    for (int t = 0; ok && t < threads; ++t) {
        job *j = &jobs[t];
        j->x = x; j->y = y; j->z = z; j->M = M;
        j->near_f = near_f; j->far_f = far_f; j->W = W; j->H = H;
        j->i0 = n * (uint64_t)t / (uint64_t)threads;
        j->i1 = n * (uint64_t)(t + 1) / (uint64_t)threads;
        j->own = bufs[t];
        j->all = bufs;
        j->nthreads = threads;
        j->out = keys;
        j->p0 = npx * t / threads;
        j->p1 = npx * (t + 1) / threads;
        if (pthread_create(&tid[t], NULL, render_job, j) != 0) { ok = 0; break; }
        ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    started = 0;
    for (int t = 0; ok && t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, merge_job, &jobs[t]) != 0) { ok = 0; break; }
        ++started;
    }
    for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    for (int t = 0; bufs && t < threads; ++t) free(bufs[t]);
    free(bufs);
    free(jobs);
    free(tid);
    return ok ? 0 : -1;
}
