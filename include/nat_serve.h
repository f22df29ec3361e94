/*
 * nat_serve.h -- C ABI of the served form of libnat_bem.so: a request server
 * that keeps meshes resident, admits Monte-Carlo and dense solves against a
 * fixed HBM budget and batches them continuously.  The solves are those of
 * nat_bem.h (Section 4.1.1 for the Monte-Carlo estimate, Section 4 and 4.1
 * for the dense Burton-Miller BEM); the server adds only scheduling, so a
 * served result is bit for bit the result of the same request run alone
 * through nat_mcbem_estimate, or through nat_bem_assemble + nat_bem_solve.
 *
 * Model
 *  - At creation the server allocates one arena of hbm_budget bytes from
 *    its context (charged to the context's budget) and starts n_slots
 *    worker threads, each with its own non-blocking HIP stream.  No device
 *    memory is allocated afterwards: every batch runs in a block carved from
 *    the arena, so the server's device use never exceeds the budget.
 *  - Requests queue in arrival order.  A free worker takes the oldest
 *    request and adds later Monte-Carlo requests with the same Neumann
 *    layout, in arrival order, while the batch has at most max_batch
 *    requests and its workspace fits a free block of the arena; it then runs
 *    the batch as one nat_mcbem_estimate_batch on its stream.  A dense
 *    request runs alone.  Batches of different workers overlap on the
 *    device, and the oldest request waits only for a free worker and room in
 *    the arena (continuous batching).
 *  - Submission validates the request on the host and rejects it with
 *    NAT_E_BUDGET when its workspace alone exceeds the budget.
 *  - The caller owns every buffer a request points to and keeps it valid and
 *    unchanged until nat_server_wait has returned its result (or the
 *    request was cancelled).
 *  - All functions may be called from any host thread.  While a server
 *    exists, its workers use the context alongside the caller's thread.
 */
#ifndef NAT_SERVE_H
#define NAT_SERVE_H

#include "nat_bem.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nat_server nat_server;

typedef enum {
    NAT_REQ_MCBEM = 0, /* Monte-Carlo estimate at query points (nat_mcbem_estimate)      */
    NAT_REQ_DENSE = 1  /* dense BEM at the triangle centroids (nat_bem_assemble + solve) */
} nat_request_kind;

typedef struct {
    int32_t n_slots;          /* worker threads / streams, 1 .. 16                         */
    int32_t max_batch;        /* requests per Monte-Carlo batch, 1 .. 4096                 */
    size_t hbm_budget;        /* arena bytes, > 0                                          */
    nat_mc_opts mc;           /* options of Monte-Carlo requests (layout is per request)   */
    double dense_tol;         /* GMRES tolerance of dense requests, > 0                    */
    int32_t dense_max_iter;   /* 1 .. 1000                                                 */
    int32_t dense_burton_miller; /* nonzero: beta = i/k; 0: conventional equation          */
} nat_server_opts;

/* 4 slots, batches of up to 64, a 16 GiB arena, nat_mc_opts_default(), and
 * dense solves with tol 1e-6, at most 200 iterations, Burton-Miller on. */
void nat_server_opts_default(nat_server_opts* opts);

typedef struct {
    int32_t kind;             /* nat_request_kind                                          */
    int32_t layout;           /* nat_neumann_layout of v_n                                 */
    nat_mesh* mesh;           /* a mesh of the server's context                            */
    int32_t n_modes;          /* 1 .. 4096                                                 */
    int32_t n_queries;        /* Monte-Carlo: Q >= 0; dense: ignored                       */
    const double* k;          /* host double[n_modes]; copied at submission                */
    const double* v_n;        /* device complex [n_modes][n_vertices or n_tris]            */
    const int32_t* q_tri;     /* Monte-Carlo: device int32[Q]                              */
    const double* q_bary;     /* Monte-Carlo: device double[Q][2]                          */
    int32_t n_samples;        /* Monte-Carlo: N >= 2                                       */
    int32_t reserved;         /* ignored                                                   */
    uint64_t seed;            /* Monte-Carlo sample seed                                   */
    double* p_out;            /* device complex: Monte-Carlo [n_modes][Q];
                                 dense [n_modes][n_tris] at the centroids                  */
    nat_solve_report* report; /* host [n_modes] or NULL; written before the result is
                                 returned by nat_server_wait                               */
} nat_request;

typedef struct {
    int32_t status;     /* the request's outcome: NAT_OK, NAT_E_NOCONV (results written),
                           NAT_E_INVALID, NAT_E_BUDGET, NAT_E_HIP, NAT_E_CANCELLED         */
    int32_t batch_size; /* requests in the batch it ran in                                 */
    int32_t slot;       /* worker that ran it, -1 if it never ran                          */
    int32_t max_iters;  /* largest GMRES iteration count over its modes                    */
    int64_t batch_id;   /* batches numbered from 1 in start order                          */
    double queue_ms;    /* start - submission (host monotonic clock)                       */
    double run_ms;      /* completion - start                                              */
    double latency_ms;  /* completion - submission                                         */
} nat_request_result;

typedef struct {
    int64_t submitted;
    int64_t completed;
    int64_t cancelled;
    int64_t batches;
    int64_t max_batch_seen;  /* most requests in one batch                                */
    int32_t max_concurrent;  /* most batches running at once                              */
    int32_t reserved;
    size_t peak_bytes;       /* most arena bytes in use at once                           */
    size_t budget;           /* arena bytes                                               */
} nat_server_stats;

/* Start a server on ctx.  NAT_E_BUDGET if the arena does not fit the
 * context's budget. */
nat_status nat_server_create(nat_ctx* ctx, const nat_server_opts* opts, nat_server** out);
/* Queue a request; *ticket identifies it.  NAT_E_INVALID (nothing queued)
 * if an argument fails validation, NAT_E_BUDGET if its workspace alone
 * exceeds the arena. */
nat_status nat_server_submit(nat_server* srv, const nat_request* req, uint64_t* ticket);
/* Wait up to timeout_ms (negative: without limit) for the request to end.
 * When it has, fills *res (may be NULL), forgets the ticket and returns the
 * request's status; NAT_E_PENDING if it is still queued or running after the
 * timeout; NAT_E_INVALID for a ticket the server does not hold. */
nat_status nat_server_wait(nat_server* srv, uint64_t ticket, double timeout_ms,
                           nat_request_result* res);
/* Remove a request that has not started: NAT_OK, and its wait returns
 * NAT_E_CANCELLED; NAT_E_INVALID if it has started, ended or is unknown. */
nat_status nat_server_cancel(nat_server* srv, uint64_t ticket);
nat_status nat_server_stats_read(nat_server* srv, nat_server_stats* out);
/* Cancel what is queued, let running batches finish, stop the workers and
 * release the arena. */
void nat_server_destroy(nat_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* NAT_SERVE_H */
