/* Plain C client of the generalized-request calls in include/mdt.h (no GPU
 * work): completion by a poll callback inside mdt_test, by one wait callback
 * for a whole group inside mdt_waitall, and by another thread; query and
 * free run once; cancel and callback error codes.  Exit status 0 on
 * success. */
#include <pthread.h>
#include <stdio.h>
#include <string.h>
#include <time.h>

#include "mdt.h"

#define CHECK(cond)                                                                  \
    do {                                                                             \
        if (!(cond)) {                                                               \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            return 1;                                                                \
        }                                                                            \
    } while (0)

typedef struct task {
    mdt_request req;
    int polls;       /* poll_fn calls so far */
    int finish_at;   /* poll_fn completes the request on this call */
    int queried, freed, cancelled, cancel_complete;
    int query_rc;    /* what query_fn returns */
    int poll_rc;     /* what poll_fn returns (until cleared) */
} task;

static int query_fn(void *s)
{
    task *t = (task *)s;
    t->queried++;
    return t->query_rc;
}

static int free_fn(void *s)
{
    ((task *)s)->freed++;
    return 0;
}

static int cancel_fn(void *s, int complete)
{
    task *t = (task *)s;
    t->cancelled++;
    t->cancel_complete = complete;
    return 0;
}

static int poll_fn(void *s)
{
    task *t = (task *)s;
    if (t->poll_rc) return t->poll_rc;
    if (++t->polls == t->finish_at) mdt_grequest_complete(t->req);
    return 0;
}

/* one call per group: completes every task it is given */
static int wait_calls, wait_last_count;
static double wait_last_timeout;
static task *wait_seen[8];
static int wait_fn(int count, void *const *states, double timeout)
{
    wait_calls++;
    wait_last_count = count;
    wait_last_timeout = timeout;
    for (int i = 0; i < count; i++) {
        task *t = (task *)states[i];
        if (i < 8) wait_seen[i] = t;
        mdt_grequest_complete(t->req);
    }
    return 0;
}

static void *completer(void *arg)
{
    struct timespec ts = {0, 20 * 1000 * 1000};
    nanosleep(&ts, NULL);
    mdt_grequest_complete(((task *)arg)->req);
    return NULL;
}

static int start(task *t, mdt_grequest_poll_fn poll, mdt_grequest_wait_fn wait)
{
    return mdt_grequest_start(query_fn, free_fn, cancel_fn, poll, wait, t, &t->req);
}

int main(void)
{
    task a;
    int flag = -1;

    /* poll-driven: not done until poll_fn completes it on its 3rd call */
    memset(&a, 0, sizeof a);
    a.finish_at = 3;
    CHECK(start(&a, poll_fn, NULL) == MDT_SUCCESS && a.req != MDT_REQUEST_NULL);
    CHECK(mdt_test(&a.req, &flag) == MDT_SUCCESS && flag == 0 && a.polls == 1);
    CHECK(mdt_test(&a.req, &flag) == MDT_SUCCESS && flag == 0 && a.polls == 2);
    CHECK(a.queried == 0 && a.freed == 0);
    CHECK(mdt_test(&a.req, &flag) == MDT_SUCCESS && flag == 1 && a.polls == 3);
    CHECK(a.req == MDT_REQUEST_NULL && a.queried == 1 && a.freed == 1);
    CHECK(mdt_test(&a.req, &flag) == MDT_SUCCESS && flag == 1); /* NULL counts as complete */

    /* mdt_wait polls until done */
    memset(&a, 0, sizeof a);
    a.finish_at = 50;
    CHECK(start(&a, poll_fn, NULL) == MDT_SUCCESS);
    CHECK(mdt_wait(&a.req) == MDT_SUCCESS && a.req == MDT_REQUEST_NULL && a.polls == 50 && a.freed == 1);

    /* a poll error ends the call and leaves the request valid */
    memset(&a, 0, sizeof a);
    a.finish_at = 1;
    a.poll_rc = 77;
    CHECK(start(&a, poll_fn, NULL) == MDT_SUCCESS);
    flag = -1;
    CHECK(mdt_test(&a.req, &flag) == 77 && flag == -1 && a.req != MDT_REQUEST_NULL);
    CHECK(mdt_wait(&a.req) == 77 && a.req != MDT_REQUEST_NULL && a.freed == 0);
    a.poll_rc = 0;
    CHECK(mdt_wait(&a.req) == MDT_SUCCESS && a.req == MDT_REQUEST_NULL && a.freed == 1);

    /* query_fn's code is returned by the call that frees the request */
    memset(&a, 0, sizeof a);
    a.finish_at = 1;
    a.query_rc = 55;
    CHECK(start(&a, poll_fn, NULL) == MDT_SUCCESS);
    CHECK(mdt_wait(&a.req) == 55 && a.req == MDT_REQUEST_NULL && a.queried == 1 && a.freed == 1);

    /* cancel reports whether the task already completed; completing twice
     * is an error */
    memset(&a, 0, sizeof a);
    CHECK(start(&a, NULL, NULL) == MDT_SUCCESS);
    CHECK(mdt_cancel(a.req) == MDT_SUCCESS && a.cancelled == 1 && a.cancel_complete == 0);
    CHECK(mdt_grequest_complete(a.req) == MDT_SUCCESS);
    CHECK(mdt_grequest_complete(a.req) == MDT_ERR_STATE);
    CHECK(mdt_cancel(a.req) == MDT_SUCCESS && a.cancelled == 2 && a.cancel_complete == 1);
    CHECK(mdt_wait(&a.req) == MDT_SUCCESS && a.freed == 1);

    /* no callbacks: another thread completes it while mdt_wait blocks */
    memset(&a, 0, sizeof a);
    CHECK(start(&a, NULL, NULL) == MDT_SUCCESS);
    pthread_t th;
    CHECK(pthread_create(&th, NULL, completer, &a) == 0);
    CHECK(mdt_wait(&a.req) == MDT_SUCCESS && a.req == MDT_REQUEST_NULL && a.freed == 1);
    pthread_join(th, NULL);

    /* waitall: one wait_fn call for the group that shares it, with no time
     * limit when nothing else needs polling */
    task g[4];
    mdt_request reqs[6];
    memset(g, 0, sizeof g);
    for (int i = 0; i < 4; i++) CHECK(start(&g[i], poll_fn, wait_fn) == MDT_SUCCESS);
    reqs[0] = g[0].req;
    reqs[1] = MDT_REQUEST_NULL;
    reqs[2] = g[1].req;
    reqs[3] = g[2].req;
    reqs[4] = g[3].req;
    wait_calls = 0;
    CHECK(mdt_waitall(5, reqs) == MDT_SUCCESS);
    CHECK(wait_calls == 1 && wait_last_count == 4 && wait_last_timeout < 0);
    CHECK(wait_seen[0] == &g[0] && wait_seen[1] == &g[1] && wait_seen[2] == &g[2] && wait_seen[3] == &g[3]);
    for (int i = 0; i < 5; i++) CHECK(reqs[i] == MDT_REQUEST_NULL);
    for (int i = 0; i < 4; i++) CHECK(g[i].queried == 1 && g[i].freed == 1 && g[i].polls == 0);

    /* mixed: a wait_fn group waits a bounded time while a poll-only task and
     * a task completed by another thread make progress */
    task p, q;
    memset(g, 0, sizeof g);
    memset(&p, 0, sizeof p);
    memset(&q, 0, sizeof q);
    p.finish_at = 5;
    CHECK(start(&g[0], NULL, wait_fn) == MDT_SUCCESS);
    CHECK(start(&p, poll_fn, NULL) == MDT_SUCCESS);
    CHECK(start(&q, NULL, NULL) == MDT_SUCCESS);
    CHECK(start(&g[1], NULL, wait_fn) == MDT_SUCCESS);
    reqs[0] = g[0].req;
    reqs[1] = p.req;
    reqs[2] = q.req;
    reqs[3] = g[1].req;
    wait_calls = 0;
    CHECK(pthread_create(&th, NULL, completer, &q) == 0);
    CHECK(mdt_waitall(4, reqs) == MDT_SUCCESS);
    pthread_join(th, NULL);
    CHECK(wait_calls == 1 && wait_last_count == 2 && wait_last_timeout > 0);
    CHECK(p.polls == 5 && p.freed == 1 && q.freed == 1 && g[0].freed == 1 && g[1].freed == 1);
    for (int i = 0; i < 4; i++) CHECK(reqs[i] == MDT_REQUEST_NULL);

    /* host cost of one request's life: start, one mdt_test whose poll
     * completes it, query and free */
    struct timespec t0, t1;
    const int reps = 200000;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int i = 0; i < reps; i++) {
        memset(&a, 0, sizeof a);
        a.finish_at = 1;
        flag = 0;
        if (start(&a, poll_fn, NULL) != MDT_SUCCESS || mdt_test(&a.req, &flag) != MDT_SUCCESS || !flag) return 1;
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    printf("grequest lifecycle %.1f ns\n", ((t1.tv_sec - t0.tv_sec) * 1e9 + (t1.tv_nsec - t0.tv_nsec)) / reps);

    /* argument errors */
    CHECK(mdt_grequest_start(NULL, NULL, NULL, NULL, NULL, NULL, NULL) == MDT_ERR_ARG);
    CHECK(mdt_grequest_complete(MDT_REQUEST_NULL) == MDT_ERR_ARG);
    CHECK(mdt_cancel(MDT_REQUEST_NULL) == MDT_ERR_ARG);
    CHECK(mdt_waitall(-1, reqs) == MDT_ERR_ARG);
    printf("grequest ok\n");
    return 0;
}
