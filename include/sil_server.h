/*
 * sil_server.h -- continuous-batching request server over libsil's batched
 * labeller (arXiv 2403.13135, section III-B "Scaling Auto-labeling": the
 * paper scales the per-image labelling with a process pool and a PySpark
 * map over images; here scenes of uneven size share GPU launches).
 *
 * Model:
 *   - A request names a scene (planar [nbands][H][pitch]), resident on the
 *     device, or in host memory with SIL_REQ_HOST_SCENE (page-locked memory,
 *     e.g. hipHostMalloc, for the copy to overlap the GPU's work).
 *   - Its outputs (label plane [H][label_pitch], rows of W labels starting on
 *     128-byte boundaries, and per-chip counts [ncy][ncx][3]) and, for a host
 *     scene, a copy of its three selected bands ([3][H][pitch]) are placed in
 *     an HBM arena of fixed size allocated at creation.  Requests are admitted
 *     first-in first-out when those bytes fit in the free arena space; the
 *     head of the queue is never overtaken.  A host scene's bands are copied
 *     into the arena at admission, on a copy stream, and its launches wait for
 *     that copy.
 *   - Admitted requests' chips are labelled by sil_label_batch launches of at
 *     most `max_chips_per_launch` chips over at most SIL_BATCH_MAX_JOBS
 *     requests, oldest first.  A large scene spans several launches; requests
 *     that arrive while launches run join the next launch.  Launches go
 *     round-robin to `nstreams` HIP streams (default priority).
 *   - A request completes when the last launch holding one of its chips has
 *     completed; its completion time is that launch's GPU event.
 *   - Outputs stay valid until sil_server_release; release only after every
 *     piece of work reading them has completed.
 *
 * Threading: a server is driven by one host thread.  Results are bit-exact
 * and independent of the mix (each chip's result depends only on its scene).
 *
 * Resource use: sil_server_create allocates the arena (hipMalloc), the
 * streams (compute and copy) and two event pools (launches; host-scene
 * copies, one per admitted request whose launches are not all enqueued yet,
 * at most 256); nothing is allocated per request.
 */
#ifndef SIL_SERVER_H
#define SIL_SERVER_H

#include <stdint.h>

#include "sil.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sil_server sil_server;

typedef struct sil_server_config {
  uint64_t arena_bytes;          /* HBM for request outputs, > 0 */
  int32_t max_chips_per_launch;  /* continuous-batching granularity, >= 1 (e.g. 4096) */
  int32_t max_inflight;          /* launches enqueued ahead of completion, 1..64 */
  int32_t nstreams;              /* compute streams, 1..8 */
  int32_t max_queue;             /* submitted-but-unadmitted requests, >= 1 */
} sil_server_config;

#define SIL_REQ_HOST_SCENE 1u /* sil_request.flags: the scene is in host memory */

typedef struct sil_request {
  const void* scene;  /* [nbands][H][pitch] of params.dtype, on the device (or in host memory
                         with SIL_REQ_HOST_SCENE); must stay valid until done */
  int32_t nbands;
  int32_t sel[3];
  int32_t H, W;
  int64_t pitch;
  uint64_t tag;       /* caller's id, unique among live requests */
  uint32_t flags;     /* 0 or SIL_REQ_HOST_SCENE */
  uint32_t pad;
} sil_request;

typedef struct sil_completion {
  uint64_t tag;
  uint8_t* labels;    /* device, [H][label_pitch], valid until sil_server_release(tag) */
  uint32_t* hist;     /* device, [ceil(H/chip)][ceil(W/chip)][3] */
  int32_t H, W;
  int32_t launches;   /* launches that held chips of this request */
  int32_t label_pitch; /* bytes between label rows: W rounded up to a multiple of 128 */
  double t_submit_ms; /* host clock at submit, ms since creation */
  double t_admit_ms;  /* host clock at admission */
  double t_done_ms;   /* GPU completion time, ms since creation */
} sil_completion;

typedef struct sil_server_stats {
  uint64_t submitted, admitted, completed, released, cancelled;
  uint64_t launches, chips;
  uint64_t arena_used, arena_peak;
  int32_t queued, active, inflight, pad;
} sil_server_stats;

/* Defaults: 4 GiB arena, 4096 chips per launch, 4 in flight, 2 streams,
 * queue of 65536. */
void sil_server_config_default(sil_server_config* c);

/* Create a server for parameters `p` (filter = 1, patch = chip; copied).
 * SIL_EINVAL on bad arguments, SIL_EUNSUPPORTED for parameters the batched
 * labeller does not take, SIL_EDEVICE if the arena, streams or events
 * cannot be created. */
int sil_server_create(const sil_params* p, const sil_server_config* cfg, sil_server** out);

/* Queue a request (host only, O(1)).  SIL_EINVAL on bad arguments (unknown
 * flags included) or a request whose arena bytes (outputs, plus the copied
 * bands of a host scene) can never fit the arena; SIL_EUNSUPPORTED when the
 * queue is full. */
int sil_server_submit(sil_server* s, const sil_request* r);

/* Admit queued requests into free arena space and enqueue launches while
 * fewer than max_inflight are outstanding.  Non-blocking.  *n_launched
 * (nullable) receives the number of launches enqueued. */
int sil_server_pump(sil_server* s, int32_t* n_launched);

/* Collect up to `max` completed requests (non-blocking; retires finished
 * launches first).  *n receives the number written to out[]. */
int sil_server_poll(sil_server* s, sil_completion* out, int32_t max, int32_t* n);

/* Return a completed request's output space to the arena.  SIL_EINVAL if
 * `tag` is not a completed, unreleased request. */
int sil_server_release(sil_server* s, uint64_t tag);

/* Withdraw a request that is still queued (not yet admitted): it will never
 * run or complete, and its tag may be reused.  SIL_EINVAL if `tag` is unknown;
 * SIL_EUNSUPPORTED if it was already admitted (its chips may be on the GPU:
 * wait for its completion and release it instead). */
int sil_server_cancel(sil_server* s, uint64_t tag);

/* Queue-wait timeout: withdraw, oldest first, the queued requests that have
 * waited more than max_wait_ms since submission (at most `max` of them) and
 * write their tags to tags[]; *n receives how many.  Admitted requests are
 * never withdrawn.  SIL_EINVAL on NULL pointers or a negative wait. */
int sil_server_expire(sil_server* s, double max_wait_ms, uint64_t* tags, int32_t max,
                      int32_t* n);

/* Block until every enqueued launch has completed (does not admit). */
int sil_server_drain(sil_server* s);

int sil_server_get_stats(const sil_server* s, sil_server_stats* out);

/* The server's host clock: ms since creation (the time base of sil_completion). */
double sil_server_clock_ms(const sil_server* s);

/* Play a request trace natively: request i is submitted once the clock
 * reaches start + arrival_ms[i] (arrival_ms non-decreasing), the server is
 * pumped and polled until all n requests have completed, and out[i] receives
 * request i's completion (matched by tag; tags must be unique).  With
 * release != 0 each request's outputs are released as soon as it completes
 * (their pointers in out[] are then stale); otherwise the caller releases.
 * *start_ms (nullable) receives the trace start on the server clock.
 * Returns SIL_EUNSUPPORTED if the queue overflows, or if with release = 0
 * the kept outputs fill the arena so that the next request can never be
 * admitted (nothing left running). */
int sil_server_run(sil_server* s, const sil_request* reqs, const double* arrival_ms, int32_t n,
                   int32_t release, sil_completion* out, double* start_ms);

/* Free everything (waits for outstanding launches first). */
int sil_server_destroy(sil_server* s);

#ifdef __cplusplus
}
#endif
#endif
