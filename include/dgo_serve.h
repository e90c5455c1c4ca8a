/*
 * dgo serving loop -- continuous batching of assembly-and-solve requests.
 *
 * Each request is one triangle mesh (positions and faces), k right-hand sides
 * f (nV x k) and asks for u after a fixed number of Jacobi-PCG iterations on
 * (alpha M + beta K) u = M f, where K and M are assembled from the request's
 * own positions (the operators of the MCF application, Sec. 7.1, applied in
 * the linear solves of Sec. 5.2). This is a system form around the paper's
 * method; the paper has no serving component.
 *
 * Requests are admitted in arrival order when a slot is free and their HBM
 * footprint fits the server's budget; admitted requests join the running
 * batch at the next tick, so requests of uneven size share every launch
 * (continuous batching). All state stays on the device until the result is
 * copied back. A request's arithmetic does not depend on the other requests
 * in the batch: its result is bitwise the same alone or in any mix.
 *
 * Threading: submit, wait, stats may be called from any host thread. The
 * server runs its own scheduler and preparation threads. Host buffers of a
 * request must stay valid until dgo_server_wait reports it finished.
 */
#ifndef DGO_SERVE_H
#define DGO_SERVE_H

#include "dgo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgo_server dgo_server;

typedef struct {
    int32_t max_slots;        /* requests in the batch at once, 1..256 */
    int32_t cg_iters;         /* PCG iterations per request (fixed, no early exit) */
    int32_t cg_chunk;         /* iterations per tick (one graph replay) */
    int32_t batched;          /* 1: continuous batching; 0: one request at a time,
                                 each with its own per-mesh launches (baseline) */
    int64_t hbm_budget_bytes; /* device memory reserved for requests at create */
    double alpha, beta;       /* operator alpha M + beta K */
    int32_t prep_threads;     /* threads that upload and build topology, >= 1 */
    int32_t pad;
} dgo_server_opts;

typedef struct {
    int32_t nV;         /* vertices */
    int32_t k;          /* right-hand sides, 1..16 */
    int64_t nF;         /* triangles */
    const int32_t *h_F; /* host, nF x 3 */
    const float *h_X;   /* host, nV x 3 */
    const float *h_f;   /* host, nV x k (the system's right-hand side is M f) */
    float *h_u;         /* host, nV x k, receives the result */
    uint64_t user;      /* caller's tag, reported back */
} dgo_request;

typedef struct {
    int32_t status;     /* dgo_status of the request */
    int32_t slot;       /* batch slot it ran in (-1 if it never ran) */
    double t_submit;    /* seconds on the server's monotonic clock */
    double t_admit;     /* admission (memory reserved, preparation started) */
    double t_start;     /* first tick that included it */
    double t_done;      /* result copied to h_u */
    int32_t iters;      /* PCG iterations run */
    int32_t pad;
    int64_t footprint;  /* bytes reserved for it */
} dgo_req_stats;

typedef struct {
    int64_t submitted, admitted, completed, rejected, failed;
    int64_t queue_depth, active;
    int64_t hbm_in_use, hbm_peak;
    int64_t ticks;          /* scheduler ticks (graph replays) */
    int64_t max_batch;      /* most requests in one tick */
    double busy_s;          /* time with at least one request on the device */
    double now_s;           /* the server clock now */
} dgo_server_counters;

/* Create a server on the current HIP device; reserves hbm_budget_bytes of
 * device memory once (all request storage comes from it). */
dgo_status dgo_server_create(const dgo_server_opts *opts, dgo_server **out);

/* Queue a request (non-blocking). DGO_ERR_BUDGET if its footprint can never
 * fit the budget, DGO_ERR_INVALID_ARG for bad sizes, DGO_ERR_SHUTDOWN after
 * destroy started. *ticket identifies it for dgo_server_wait. */
dgo_status dgo_server_submit(dgo_server *srv, const dgo_request *req, uint64_t *ticket);

/* Wait until the request finished or timeout_s elapsed (DGO_ERR_TIMEOUT).
 * On return h_u holds the result; st (may be NULL) receives its record.
 * Returns the request's own status (DGO_OK, or why it failed). A ticket can
 * be waited for once. */
dgo_status dgo_server_wait(dgo_server *srv, uint64_t ticket, double timeout_s, dgo_req_stats *st);

dgo_status dgo_server_stats(dgo_server *srv, dgo_server_counters *out);

/* Footprint in bytes that the server reserves for a request of this shape. */
int64_t dgo_server_footprint(int32_t nV, int64_t nF, int32_t k);

/* Finish every queued and running request, then release the server. */
void dgo_server_destroy(dgo_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* DGO_SERVE_H */
