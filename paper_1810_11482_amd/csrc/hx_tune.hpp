// Launch-geometry cache of the autotuner.  Keys name the kernel family, the
// dtype, the problem size class and the step count; values are geometries.  The
// cache is process-wide, filled by the hx_tune_* entry points and persisted as
// a small JSON object (HX_TUNE_CACHE names the file).
#pragma once

#include <string>

#include "hx_internal.h"

namespace hx {

struct Ctx;

struct TuneKey {
    std::string s;
};

struct TunedGeom {
    int cpl = 0;       // 1D/2D cells per lane
    int steps = 0;     // time block
    int wpg = 0;       // waves per group
    int rows = 0;      // 2D rows per wave
    int grid = 0;      // batched: waves per CU
    int mode = 0;      // batched: chosen hx_batch_form + 1 (0 = none)
                       // (a batched propagator keeps its span_blocks in `rows`)
};

TuneKey tune_key_1d(int dtype, int64_t n, int steps, bool ghost);
TuneKey tune_key_2d(int dtype, int64_t ny, int64_t nx, int steps);
TuneKey tune_key_batched(int dtype, int64_t total_cells, int count, int steps);

bool tune_lookup(const TuneKey& k, TunedGeom* g);
void tune_store(const TuneKey& k, const TunedGeom& g);

// Default 1D geometry for a key: the tuned entry if one exists, otherwise the
// built-in heuristic.
Geom1D default_geom_1d(Ctx* c, const TuneKey& k);

int max_time_block_1d(int dtype, int cpl);

}  // namespace hx
