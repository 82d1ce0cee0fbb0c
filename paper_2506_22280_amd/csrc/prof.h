// prof.h -- opt-in stage timing with HIP events recorded on the launch stream.
#pragma once

#include "common.h"

enum ProfStage {
    PS_FFD = 0,
    PS_SETUP,
    PS_SCAN,
    PS_BIN_COUNT,
    PS_BIN_FILL,
    PS_SPLAT_FWD,
    PS_SPLAT_BWD,
    PS_CELL_SORT,
    PS_GAUSS_BWD,
    PS_COEF_GRAD,
    PS_OTHER,
    PS_COUNT
};

bool prof_on();
void prof_begin(int stage, hipStream_t s);
void prof_end(int stage, hipStream_t s);

// While one exists on a thread, that thread's launches record no stage events (for calls that
// must not create events or grow host-side lists).
struct ProfSuppress {
    ProfSuppress();
    ~ProfSuppress();
};

// stage < 0: no timing
struct ProfScope {
    int stage;
    hipStream_t s;
    ProfScope(int st, hipStream_t ss) : stage(st), s(ss)
    {
        if (stage >= 0 && prof_on()) prof_begin(stage, s);
    }
    ~ProfScope()
    {
        if (stage >= 0 && prof_on()) prof_end(stage, s);
    }
};
