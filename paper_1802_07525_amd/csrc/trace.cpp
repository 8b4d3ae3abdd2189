// trace.cpp -- optional roctx ranges around the library's host phases:
// steady solves, cell updates, coupled-loop updates, hourly model
// intervals, and the server's preparations, batch chunks and solo solves.
//
// Off unless the environment variable LBM_ROCTX is set when the first range
// opens.  "1" loads ROCm's marker library (librocprofiler-sdk-roctx.so.1,
// else the older libroctx64.so.4); any other value except "0" is the path
// of a library exporting roctxRangePushA and roctxRangePop.  The library is
// opened with dlopen and kept open until the process ends, so _lbm.so has
// no link-time dependency on it.  When the ranges are off, or the library
// cannot be opened (one message on stderr), a range costs one read of a
// pointer resolved once.  roctx ranges are per thread, so a Range is pushed
// and popped on the thread that owns it.

#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm_internal.h"

namespace {

struct Roctx {
    int (*push)(const char *) = nullptr;
    int (*pop)() = nullptr;
};

Roctx open_roctx()
{
    Roctx r;
    const char *v = getenv("LBM_ROCTX");
    if (!v || !*v || !strcmp(v, "0"))
        return r;
    void *h = nullptr;
    if (!strcmp(v, "1")) {
        h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
        if (!h)
            h = dlopen("libroctx64.so.4", RTLD_NOW | RTLD_LOCAL);
    } else {
        h = dlopen(v, RTLD_NOW | RTLD_LOCAL);
    }
    if (!h) {
        const char *why = dlerror();
        fprintf(stderr, "lbm: LBM_ROCTX=%s: cannot open the roctx library (%s); no ranges\n", v,
                why ? why : "unknown error");
        return r;
    }
    void *push = dlsym(h, "roctxRangePushA");
    void *pop = dlsym(h, "roctxRangePop");
    if (!push || !pop) {
        fprintf(stderr, "lbm: LBM_ROCTX=%s: the library lacks roctxRangePushA/roctxRangePop; no ranges\n",
                v);
        return r;
    }
    r.push = reinterpret_cast<int (*)(const char *)>(push);
    r.pop = reinterpret_cast<int (*)()>(pop);
    return r;
}

const Roctx &roctx()
{
    static const Roctx r = open_roctx(); // resolved once, thread-safe
    return r;
}

} // namespace

lbmh::Range::Range(const char *name) : on_(false)
{
    const Roctx &r = roctx();
    if (r.push) {
        r.push(name);
        on_ = true;
    }
}

lbmh::Range::~Range()
{
    if (on_)
        roctx().pop();
}
