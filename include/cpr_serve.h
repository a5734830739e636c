/*
 * cpr_serve.h - a request-serving runtime over the CPR-FGMRES solver.
 *
 * Requests are Jacobian solves of different sizes arriving over time.  The
 * server keeps each case's SETUP products (AMG hierarchy, stage-2 data) and
 * Krylov workspace resident in device memory between requests, so a request
 * that is the next Newton step of a resident case goes through
 * cpr_update_values and the adaptive-setup rule of Algorithm "ASCPR" (reuse
 * across Newton steps, Section 4) instead of a fresh SETUP.
 *
 * Continuous batching: up to max_slots requests run at once, each on its own
 * worker thread and HIP stream, so their kernels overlap on the device.  A
 * pending request starts as soon as a slot is free, its case is not already
 * running, and its device memory fits the budget (idle resident cases are
 * evicted least-recently-used first to make room).  Requests of one case run
 * in submission order.  Every kernel of a request works on that case's own
 * buffers with fixed reduction orders, so a result does not depend on which
 * other requests ran beside it.
 */
#ifndef CPR_MI355X_SERVE_H
#define CPR_MI355X_SERVE_H

#include <stdint.h>

#include "cpr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpr_server cpr_server;

typedef struct {
  int64_t case_id;  /* requests with one id are successive Newton steps of one case
                       (same sparsity pattern); a different pattern replaces the case */
  cpr_bsr A;        /* host arrays (location CPR_MEM_HOST); the caller keeps them alive
                       until cpr_server_wait has returned for this request */
  const double* b;  /* host right-hand side, 3*n_block_rows doubles, same lifetime rule */
  double* x;        /* host output, 3*n_block_rows doubles (initial guess 0) */
  double tol;       /* relative residual tolerance */
} cpr_request;

typedef struct {
  int64_t submitted, completed, rejected;
  int64_t setups, reuses, evictions;
  int64_t resident_cases, bytes_in_use, bytes_peak, budget_bytes;
} cpr_server_stats;

/* Start a server on the current HIP device with max_slots worker threads (each
 * with its own stream) and a device-memory budget in bytes for all resident
 * cases.  p: solver parameters of every case (NULL = defaults). */
cpr_status cpr_server_create(int64_t budget_bytes, int32_t max_slots, const cpr_params* p, cpr_server** out);

/* Queue a request; returns at once with a ticket.  CPR_ERR_INVALID_ARG for a
 * malformed request (checked before queueing). */
cpr_status cpr_server_submit(cpr_server* s, const cpr_request* r, int64_t* ticket);

/* Block until the request is done; then x holds the solution.  Returns the
 * request's status (CPR_ERR_OOM if it can never fit the budget), fills info
 * (may be NULL) and the latency from submission to completion in ms. */
cpr_status cpr_server_wait(cpr_server* s, int64_t ticket, cpr_solve_info* info, double* latency_ms);

cpr_status cpr_server_stats_get(cpr_server* s, cpr_server_stats* out);

/* Text of the most recent failed request ("" if none); valid until the next
 * call on s. */
const char* cpr_server_last_error(cpr_server* s);

/* Finish queued requests, stop the workers and free every resident case. */
void cpr_server_destroy(cpr_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CPR_MI355X_SERVE_H */
