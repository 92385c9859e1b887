// Host-side state behind the C-ABI handles.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <tuple>

#include "gscl.h"
#include "launch.h"

enum { CTX_INIT = 0, CTX_ACTIVE = 1, CTX_ENDED = 2, CTX_FINALIZED = 3 };

struct gscl_ctx {
    uint32_t magic;
    int device;
    int state;
    hipStream_t stream;
    double* partials;      // per-block reduction partials
    int64_t partial_cap;   // doubles
    double* result;        // device slots for reduction results
    bool capturing;
    std::map<std::tuple<int, int, int64_t, int64_t, int64_t>, gk::TileCfg> tiles;
};

struct gscl_grid {
    uint32_t magic;
    gscl_ctx* ctx;
    gscl_grid_desc d;      // pitches resolved
    void* ptr;
    size_t bytes;
};

struct gscl_graph {
    uint32_t magic;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

constexpr uint32_t CTX_MAGIC = 0x47534331u, GRID_MAGIC = 0x47534332u, GRAPH_MAGIC = 0x47534333u,
                   BATCH_MAGIC = 0x47534334u;

// error helpers (thread-local message)
int gscl_fail(int code, const char* fmt, ...);
int gscl_hip_fail(hipError_t e, const char* what);
#define GSCL_HIP(call)                                    \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return gscl_hip_fail(e_, #call); \
    } while (0)

size_t dtype_size(int dt);
gk::Geo geo_of(const gscl_grid* g);
int ensure_partials(gscl_ctx* c, int64_t nblocks);
gk::TileCfg pick_tile(gscl_ctx* c, int kind, int dtype, const gscl_grid_desc& d);
bool ctx_ok(const gscl_ctx* c);
bool grid_ok(const gscl_grid* g);
