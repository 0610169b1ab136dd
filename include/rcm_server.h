/*
 * rcm_server.h -- a request-serving engine for Reverse Cuthill-McKee
 * orderings on one GPU, as a C ABI.
 *
 * Each request is one ordering as defined in rcm.h: the operation of the
 * paper "The Reverse Cuthill-McKee Algorithm in Distributed-Memory" (Azad,
 * Jacquelin, Buluc, Ng), Section I (find P so that P A P^T has a small
 * bandwidth), computed per Algorithms 2 and 3 with the deterministic ties
 * documented in rcm.h.  The result of a request is bit-identical to what
 * rcm_order_ex returns for the same pattern alone.
 *
 * What the engine adds around the per-call library:
 *   - a device memory arena of a fixed budget, allocated once at creation;
 *     the CSR, results and workspace of requests in flight live in it, so
 *     serving allocates no device memory per request;
 *   - admission by memory footprint: a request waits (first come, first
 *     served) until its footprint fits in the arena; a request whose
 *     footprint exceeds the whole budget fails alone with
 *     RCM_ERR_OUT_OF_MEMORY;
 *   - continuous batching: whenever an executor is free it takes the
 *     waiting requests from the head of the queue, as many as fit (memory,
 *     max_batch, batch_nnz_limit), and orders them in one batched call
 *     (rcm_order_batched), whose single persistent launch runs the
 *     components of all of them concurrently; a request above
 *     batch_nnz_limit, or alone in the queue, runs by itself (rcm_order_ex);
 *   - several executors, each a host thread with its own HIP stream (default
 *     priority), so that one batch's host-to-device copies overlap another
 *     batch's kernels;
 *   - per-request timestamps (submit, admission, completion) for latency
 *     percentiles.
 *
 * A malformed or asymmetric request fails alone: when a batched call fails,
 * its requests are re-run one by one, so only the offending ones report the
 * error.
 *
 * Thread safety: every function may be called from any thread.
 */
#ifndef RCM_SERVER_H_
#define RCM_SERVER_H_

#include <stddef.h>
#include <stdint.h>

#include "rcm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rcm_server rcm_server;

typedef struct {
  uint64_t mem_budget_bytes; /* device arena size; 0 = auto (1 GiB)                 */
  int32_t max_batch;         /* most requests in one batched call; 0 = auto (32)     */
  int32_t executors;         /* executor threads / streams; 0 = auto (2), at most 8 */
  int64_t batch_nnz_limit;   /* requests with more CSR entries run alone; 0 = auto
                                (no limit: one persistent launch orders the
                                components of all batched requests concurrently,
                                which keeps the GPU busier than requests run one
                                by one)                                              */
  rcm_options order_options; /* options of every ordering (see rcm.h); the server
                                keeps its own copy of tuning_file               */
} rcm_server_config;

/* Outcome of one request. Times are seconds on the host's steady clock,
   relative to the server's creation. */
typedef struct {
  int32_t status;      /* rcm_status of the ordering itself                         */
  int32_t batch_size;  /* requests in the call that ordered it (1 = alone)          */
  rcm_stats stats;     /* as rcm_order_ex reports them                               */
  double t_submit;     /* rcm_server_submit returned                                 */
  double t_admit;      /* an executor took it (memory reserved)                      */
  double t_done;       /* perm_out written, request complete                         */
} rcm_request_result;

typedef struct {
  int64_t submitted, completed, failed; /* requests                                 */
  int64_t batches;                       /* device calls made (batched or alone)     */
  int64_t retried_alone;                 /* requests re-run alone after a batch failed */
  int64_t max_batch_seen;
  uint64_t bytes_in_flight;              /* arena bytes reserved now                 */
  uint64_t peak_bytes_in_flight;         /* highest reservation so far               */
  uint64_t mem_budget_bytes;
} rcm_server_counters;

/* Fill *cfg with the defaults (all zero = auto). */
void rcm_server_default_config(rcm_server_config* cfg);

/* Device bytes a request of n vertices and nnz entries reserves while in
   flight when it runs alone (CSR, perm, iperm and workspace); batched
   requests reserve the same order of magnitude. */
uint64_t rcm_server_request_bytes(int32_t n, int64_t nnz);

/* Create a server on the current HIP device: allocates the arena and
   starts the executors.  Errors: RCM_ERR_INVALID_ARGUMENT (bad config or
   options, NULL out), RCM_ERR_OUT_OF_MEMORY (arena allocation failed),
   RCM_ERR_HIP. */
rcm_status rcm_server_create(const rcm_server_config* cfg, rcm_server** out);

/* Queue one ordering.  rowptr_host (int32[n+1]), colidx_host (int32[nnz])
   and perm_out_host (int32[n], receives new -> old) are HOST pointers owned
   by the caller, which keeps them valid and unmodified until the request is
   complete (rcm_server_wait or a done poll).  n == 0 completes at once.
   Returns RCM_ERR_INVALID_ARGUMENT for n < 0, nnz < 0 or NULL pointers; any
   other failure is reported by the request's own status. */
rcm_status rcm_server_submit(rcm_server* srv, int32_t n, int64_t nnz, const int32_t* rowptr_host,
                             const int32_t* colidx_host, int32_t* perm_out_host,
                             int64_t* ticket_out);

/* Non-blocking: *done = 1 when the request is complete. */
rcm_status rcm_server_poll(rcm_server* srv, int64_t ticket, int32_t* done);

/* Block until the request is complete (timeout_ms < 0: no limit), then
   write its result and release the ticket.  Returns RCM_ERR_ABORTED on a
   timeout (the ticket stays valid), RCM_ERR_INVALID_ARGUMENT for an unknown
   ticket. */
rcm_status rcm_server_wait(rcm_server* srv, int64_t ticket, int64_t timeout_ms,
                           rcm_request_result* result);

rcm_status rcm_server_counters_get(rcm_server* srv, rcm_server_counters* out);

/* Stop accepting requests, finish the queued ones, stop the executors and
   free the arena.  Results not yet collected are discarded. */
void rcm_server_destroy(rcm_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* RCM_SERVER_H_ */
