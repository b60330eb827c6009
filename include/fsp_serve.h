/*
 * fsp_serve.h -- a serving engine over the free-space Poisson solver of fsp.h
 * (continuous batching of independent solve requests on one GPU).
 *
 * No passage of the paper defines this layer: every request is one fsp_solve
 * (the result Section 2.2 defines, with the Green's function of Sections
 * 2.2-2.4).  Two statements of the paper shape it: the precomputed transform
 * of G2 is reused by every solve on the same grid and box (Section 2.3), and a
 * grid fitted to a changing particle bunch needs it recomputed whenever the box
 * changes (Section 1); here the transforms are cached per (Green's function,
 * grid, box, alpha, precision) and computed on a miss.
 *
 * The engine runs on the calling host thread inside fsp_server_run: requests
 * are released at their arrival times (host clock), queued in arrival order,
 * and admitted while a launch slot (a HIP stream of the engine) is free and
 * the device bytes the engine holds stay within its budget.  An admitted
 * request of the queue's head takes with it up to max_fold - 1 queued requests
 * of the same grid and precision (any Green's function and box), and they are
 * solved by shared kernel launches.  A Green's transform missing from the
 * cache is computed on the engine's refresh stream; the solves that read it
 * wait for it on the device, and its time is reported with them.
 *
 * Bytes held (the budget covers all of them): the cached Green's buffers, the
 * solve workspaces (kept in a pool per grid and precision and reused), and the
 * transient buffers of refreshes in flight.  When an admission would exceed
 * the budget, idle workspaces and cached transforms no solve is using are
 * freed, least recently used first.  A request that would not fit an empty
 * engine is rejected (FSP_ERR_OUT_OF_MEMORY in its result).  rho and phi are
 * the caller's device arrays and are not counted.
 */
#ifndef FSP_SERVE_H_
#define FSP_SERVE_H_

#include <stddef.h>

#include "fsp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsp_server_s* fsp_server;

typedef struct {
  double t_arrival;   /* seconds after fsp_server_run starts (scaled by time_scale) */
  int n[3];           /* grid points per axis (fsp_plan_desc.n)                      */
  int greens;         /* fsp_greens                                                   */
  int prec;           /* fsp_prec                                                     */
  double lo[3];       /* box lower corner                                             */
  double hi[3];       /* box upper corner                                             */
  double alpha;       /* Vico-Greengard window factor; 0 -> 1.1                       */
  const void* rho;    /* device array [n0][n1][n2] of the precision                   */
  void* phi;          /* device array for the result; may equal rho                   */
} fsp_request;

typedef struct {
  double t_arrival;   /* arrival time on the run's clock, seconds (scaled)            */
  double t_admit;     /* host time of its admission, seconds                          */
  double t_done;      /* device time its launch completed, seconds                    */
  double t_seen;      /* host time the engine saw the completion, seconds             */
  float refresh_ms;   /* the Green's refresh it waited for, 0 on a cache hit          */
  int status;         /* FSP_OK; FSP_ERR_OUT_OF_MEMORY if rejected; else its error   */
  int slot;           /* launch slot (stream) it ran on                               */
  int launch_size;    /* requests solved by its launch                                */
} fsp_request_result;

typedef struct {
  size_t budget_bytes;         /* the budget                                          */
  size_t peak_held_bytes;      /* most bytes held at once (never above the budget)    */
  size_t held_bytes;           /* bytes held when the run ended (cache and pool)      */
  long long launches;          /* solve launches                                      */
  long long refreshes;         /* Green's transforms computed                         */
  long long evictions;         /* buffers freed to make room                          */
  long long rejected;          /* requests larger than the budget                     */
  double refresh_ms_total;     /* device time of all refreshes                        */
} fsp_server_stats;

/* An engine with `slots` launch streams (1..64), a device-byte budget and at
 * most max_fold requests per launch (1..256), on the current HIP device. */
fsp_status fsp_server_create(size_t budget_bytes, int slots, int max_fold, fsp_server* out);

/* Serve count requests (any order of t_arrival; each is released at
 * t_arrival * time_scale seconds after the start, so 0 releases all at once)
 * and fill results[i] for reqs[i].  Returns when every request is done or
 * rejected, or after max_wall_s seconds (FSP_ERR_DEVICE; unfinished requests
 * keep status FSP_ERR_NOT_READY).  Blocking; the cache and pool persist into
 * the next run.  Argument errors (a NULL pointer, a descriptor fsp_plan_create
 * rejects) are reported before anything runs. */
fsp_status fsp_server_run(fsp_server s, int count, const fsp_request* reqs, fsp_request_result* results,
                          double time_scale, double max_wall_s);

fsp_status fsp_server_get_stats(fsp_server s, fsp_server_stats* out);

/* Wait for the engine's work and free everything it holds. */
fsp_status fsp_server_destroy(fsp_server s);

#ifdef __cplusplus
}
#endif

#endif /* FSP_SERVE_H_ */
