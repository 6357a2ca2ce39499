/*
 * hullf_server.h -- C ABI of the request loop: continuous batching of convex
 * hull requests on one GPU.
 *
 * Each request is one host point set whose hull (Algorithm 1 of arXiv
 * 2303.10581, Sec. 3.1-3.3) is wanted.  The loop, run by threads the server
 * owns:
 *  1. admits requests in arrival order while a request slot and room in the
 *     device arena are free (admission by device memory);
 *  2. copies each admitted request's points into its arena region, on two
 *     copy streams (two copies in flight; HULLF_SERVER_COPIERS=1..4 at
 *     creation sets the number), while earlier batches run;
 *  3. whenever the device is idle, launches one batched filter over every
 *     request whose points are resident (hull_filter_segments in hullf.h:
 *     extremes, inside test and compaction per request, one launch set);
 *  4. finishes each request's hull from its resident survivors
 *     (hull_from_survivors: monotone chain, Sec. 3.3) on a finisher thread
 *     and stream, then frees its arena region, while later batches run.
 * Requests that arrive while a batch runs join the next batch.  A request's
 * hull depends only on its own points: it is the same alone or in any mix
 * (hull conventions as in hullf.h).
 *
 * Threads: submit, wait and stats may be called from any host threads.
 */
#ifndef HULLF_SERVER_H
#define HULLF_SERVER_H

#include "hullf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hullf_server *hullf_server_t;

typedef struct {
    /* Points the device arena holds at once (12 bytes each: the point and
     * its survivor slot).  0 = 2^28.  A request larger than this is refused. */
    uint64_t arena_points;
    /* Requests admitted at once (slots).  0 = 1024. */
    uint32_t max_inflight;
    /* Threads finishing hulls (each with its own context and stream: the
     * device sort and chains for large survivor sets, the host chain for
     * small ones).  0 = 4. */
    uint32_t finish_threads;
    uint32_t reserved[2];
} hullf_server_config;

/* Timeline and sizes of one finished request.  Times are microseconds
 * after its submit call. */
typedef struct {
    double admitted_us;   /* slot and arena region granted */
    double resident_us;   /* points copied into device memory */
    double launched_us;   /* its batch enqueued */
    double filtered_us;   /* its batch finished (survivor counts on the host) */
    double done_us;       /* hull finished */
    uint64_t n;           /* points */
    uint64_t survivors;   /* points that passed the filter */
    uint64_t hull;        /* hull vertices */
    uint64_t batch;       /* serial number of its batch */
    uint32_t batch_requests;  /* requests in that batch */
    uint32_t status;      /* hullf_status of the request */
} hullf_request_info;

typedef struct {
    uint64_t submitted, completed;
    uint64_t batches, batched_requests;   /* launches and requests they held */
    uint64_t arena_points, arena_peak_points;
    uint32_t inflight, queued;            /* admitted / waiting for admission */
    double batch_ms;                      /* summed launch-to-finish time of the batches */
} hullf_server_counters;

/* Start a server on HIP device `device` (cfg may be NULL for defaults).
 * Allocates the arena and starts its threads.  *out is set only on
 * HULLF_OK. */
hullf_status hullf_server_create(int device, const hullf_server_config *cfg,
                                 hullf_server_t *out);

/* Finish every submitted request, stop the threads and release the server.
 * Results not yet collected are dropped.  NULL is ignored. */
void hullf_server_destroy(hullf_server_t srv);

/* Queue a request; returns at once with its id in *id.
 * h_pts: n host points; the memory must stay valid and unchanged until
 * hullf_server_wait has returned the request's result.  Page-locked memory
 * (hipHostMalloc) is copied to the device directly, other memory through the
 * server's staging buffers.  n == 0 completes at once with an empty hull.
 * Returns HULLF_EINVAL for n >= 2^32 or a null pointer, HULLF_ENOMEM if n
 * exceeds the arena. */
hullf_status hullf_server_submit(hullf_server_t srv, const hullf_pt *h_pts,
                                 uint64_t n, uint64_t *id);

/* Wait up to timeout_ms (< 0: no limit, 0: poll) for request `id`.
 * Returns HULLF_EAGAIN if it has not finished.  Otherwise returns the
 * request's status and, on HULLF_OK, writes its counter-clockwise hull
 * (indices into its h_pts) to h_hull (capacity cap) and the vertex count to
 * *h_count.  If cap is too small it returns HULLF_ECAPACITY with *h_count
 * set and keeps the result for another call; every other finished outcome
 * releases the request.  info may be NULL.  Unknown ids give HULLF_EINVAL. */
hullf_status hullf_server_wait(hullf_server_t srv, uint64_t id, int timeout_ms,
                               uint32_t *h_hull, uint64_t cap, uint64_t *h_count,
                               hullf_request_info *info);

/* Counters since creation. */
hullf_status hullf_server_stats(hullf_server_t srv, hullf_server_counters *out);

#ifdef __cplusplus
}
#endif

#endif /* HULLF_SERVER_H */
