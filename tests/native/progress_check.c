/* Plain C client of the general-progress calls in include/mdt.h (no GPU
 * work): generalized requests completed by explicit progress passes and by
 * the library's progress thread, with no test or wait call in between;
 * mdt_request_get_status reports completion without freeing; poll
 * callbacks never run on two threads at once; a poll error is returned by
 * the pass; start and stop are idempotent; a stream with no requests
 * progresses trivially.  Exit status 0 on success. */
#include <stdatomic.h>
#include <stdio.h>
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
    atomic_int polls;     /* poll_fn calls so far */
    atomic_int inside;    /* threads inside poll_fn right now */
    atomic_int overlap;   /* poll_fn found another thread inside */
    int finish_at;        /* poll_fn completes the request on this call */
    int poll_rc;          /* what poll_fn returns */
    atomic_int queried;
} task;

static int poll_fn(void *s)
{
    task *t = (task *)s;
    if (atomic_fetch_add(&t->inside, 1) != 0) atomic_fetch_add(&t->overlap, 1);
    int n = atomic_fetch_add(&t->polls, 1) + 1;
    if (n == t->finish_at) mdt_grequest_complete(t->req);
    atomic_fetch_sub(&t->inside, 1);
    return t->poll_rc;
}

static int query_fn(void *s)
{
    atomic_fetch_add(&((task *)s)->queried, 1);
    return 0;
}

static void nap_us(long us)
{
    struct timespec ts = {0, us * 1000};
    nanosleep(&ts, NULL);
}

int main(void)
{
    /* explicit general progress: three passes complete a task that needs three polls */
    task a = {0};
    a.finish_at = 3;
    CHECK(mdt_grequest_start(query_fn, NULL, NULL, poll_fn, NULL, &a, &a.req) == MDT_SUCCESS);
    int flag = -1;
    CHECK(mdt_request_get_status(a.req, &flag) == MDT_SUCCESS && flag == 0);
    for (int i = 0; i < 3; i++) CHECK(mdt_stream_progress(NULL) == MDT_SUCCESS);
    CHECK(atomic_load(&a.polls) == 3);
    CHECK(mdt_request_get_status(a.req, &flag) == MDT_SUCCESS && flag == 1);
    CHECK(a.req != MDT_REQUEST_NULL && atomic_load(&a.queried) == 0); /* not freed by get_status */
    CHECK(mdt_stream_progress(NULL) == MDT_SUCCESS && atomic_load(&a.polls) == 3); /* done: no more polls */
    CHECK(mdt_test(&a.req, &flag) == MDT_SUCCESS && flag == 1 && a.req == MDT_REQUEST_NULL);
    CHECK(atomic_load(&a.queried) == 1);

    /* a stream with no requests: progress passes do nothing */
    mdt_stream s = NULL;
    CHECK(mdt_stream_create(NULL, &s) == MDT_SUCCESS);
    CHECK(mdt_stream_progress(s) == MDT_SUCCESS);
    CHECK(mdt_start_progress_thread(s) == MDT_SUCCESS);
    CHECK(mdt_start_progress_thread(s) == MDT_SUCCESS); /* already running */
    CHECK(mdt_stop_progress_thread(s) == MDT_SUCCESS);
    CHECK(mdt_stop_progress_thread(s) == MDT_SUCCESS); /* already stopped */

    /* the progress thread completes tasks in the background while this
     * thread also tests them: polls never overlap */
    task t[4];
    for (int i = 0; i < 4; i++) {
        task z = {0};
        t[i] = z;
        t[i].finish_at = 200 + 100 * i;
        CHECK(mdt_grequest_start(query_fn, NULL, NULL, poll_fn, NULL, &t[i], &t[i].req) == MDT_SUCCESS);
    }
    CHECK(mdt_start_progress_thread(NULL) == MDT_SUCCESS);
    for (int spins = 0; spins < 200000; spins++) {
        int done = 0;
        for (int i = 0; i < 4; i++) {
            CHECK(mdt_request_get_status(t[i].req, &flag) == MDT_SUCCESS);
            done += flag;
        }
        if (done == 4) break;
        if (spins % 7 == 0) { /* tests race with the thread's polls */
            int f = 0;
            CHECK(mdt_test(&t[0].req, &f) == MDT_SUCCESS);
            if (f) CHECK(t[0].req == MDT_REQUEST_NULL);
            if (f) {
                /* completed and freed by this test: keep status queries valid */
                t[0].req = MDT_REQUEST_NULL;
            }
        }
        nap_us(20);
    }
    for (int i = 0; i < 4; i++) {
        CHECK(mdt_request_get_status(t[i].req, &flag) == MDT_SUCCESS && flag == 1);
        CHECK(atomic_load(&t[i].polls) == t[i].finish_at);
        CHECK(atomic_load(&t[i].overlap) == 0);
    }
    CHECK(mdt_stop_progress_thread(NULL) == MDT_SUCCESS);
    mdt_request all[4];
    for (int i = 0; i < 4; i++) all[i] = t[i].req;
    CHECK(mdt_waitall(4, all) == MDT_SUCCESS);
    for (int i = 1; i < 4; i++) CHECK(atomic_load(&t[i].queried) == 1);

    /* a poll error ends the pass with that code; the request stays valid */
    task e = {0};
    e.finish_at = 2;
    e.poll_rc = 77;
    CHECK(mdt_grequest_start(NULL, NULL, NULL, poll_fn, NULL, &e, &e.req) == MDT_SUCCESS);
    CHECK(mdt_stream_progress(NULL) == 77);
    CHECK(mdt_request_get_status(e.req, &flag) == MDT_SUCCESS && flag == 0);
    e.poll_rc = 0;
    CHECK(mdt_stream_progress(NULL) == MDT_SUCCESS);
    CHECK(mdt_request_get_status(e.req, &flag) == MDT_SUCCESS && flag == 1);
    CHECK(mdt_wait(&e.req) == MDT_SUCCESS && e.req == MDT_REQUEST_NULL);

    /* argument errors */
    CHECK(mdt_request_get_status(NULL, &flag) == MDT_SUCCESS && flag == 1);
    CHECK(mdt_request_get_status(NULL, NULL) == MDT_ERR_ARG);
    CHECK(mdt_stream_free(&s) == MDT_SUCCESS);
    printf("progress ok\n");
    return 0;
}
