/* roctx_stub.c -- a stand-in for ROCm's roctx marker library, for the CPU
 * tests of the library's ranges (LBM_ROCTX=<path of this library>).
 *
 * It exports the two calls the library uses, roctxRangePushA and
 * roctxRangePop, with roctx's meaning: ranges nest per thread, a push
 * returns the level it opens (0-based), a pop returns the level it closes,
 * or -1 with no range open.  It counts pushes per range name and records
 * every misuse: a pop with no range open on its thread, and a thread that
 * ends with ranges open.  At process exit it writes its counts to the file
 * that ROCTX_STUB_OUT names:
 *   pushes P / pops Q / bad_pops B / unbalanced U / max_depth D
 *   then one line "range <name> <count>" per name.                         */
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAX_NAMES 64

static pthread_mutex_t mu = PTHREAD_MUTEX_INITIALIZER;
static pthread_key_t open_key;
static pthread_once_t key_once = PTHREAD_ONCE_INIT;
static __thread int depth;
static long pushes, pops, bad_pops, unbalanced;
static int max_depth;
static char *names[MAX_NAMES];
static long counts[MAX_NAMES];
static int n_names;

/* runs when a thread that still has ranges open ends */
static void thread_end(void *v)
{
    (void)v;
    pthread_mutex_lock(&mu);
    ++unbalanced;
    pthread_mutex_unlock(&mu);
}

static void make_key(void) { pthread_key_create(&open_key, thread_end); }

int roctxRangePushA(const char *message)
{
    pthread_once(&key_once, make_key);
    const int level = depth++;
    pthread_setspecific(open_key, (void *)1);
    pthread_mutex_lock(&mu);
    ++pushes;
    if (depth > max_depth)
        max_depth = depth;
    int k = 0;
    while (k < n_names && strcmp(names[k], message) != 0)
        ++k;
    if (k == n_names && n_names < MAX_NAMES) {
        const size_t len = strlen(message) + 1;
        names[n_names] = (char *)malloc(len);
        memcpy(names[n_names++], message, len);
    }
    if (k < MAX_NAMES)
        ++counts[k];
    pthread_mutex_unlock(&mu);
    return level;
}

int roctxRangePop(void)
{
    pthread_once(&key_once, make_key);
    pthread_mutex_lock(&mu);
    if (depth == 0) {
        ++bad_pops;
        pthread_mutex_unlock(&mu);
        return -1;
    }
    ++pops;
    pthread_mutex_unlock(&mu);
    const int level = --depth;
    if (depth == 0)
        pthread_setspecific(open_key, NULL);
    return level;
}

__attribute__((destructor)) static void report(void)
{
    const char *path = getenv("ROCTX_STUB_OUT");
    if (!path)
        return;
    FILE *f = fopen(path, "w");
    if (!f)
        return;
    pthread_mutex_lock(&mu);
    /* the exiting thread's own ranges count as open too */
    fprintf(f, "pushes %ld\npops %ld\nbad_pops %ld\nunbalanced %ld\nmax_depth %d\n", pushes, pops, bad_pops,
            unbalanced + (depth != 0), max_depth);
    for (int k = 0; k < n_names; ++k)
        fprintf(f, "range %s %ld\n", names[k], counts[k]);
    pthread_mutex_unlock(&mu);
    fclose(f);
}
