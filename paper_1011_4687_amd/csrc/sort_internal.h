// Spatial ordering of evaluation points (sortpts.hip).  Not part of the C ABI.
#pragma once

#include <cstdint>

namespace envpot {

// Points with at least this many entries are evaluated in Morton order
// (not while the stream is being captured into a graph: the sort library
// may record memory-set nodes).
constexpr int64_t kSortMinPoints = 32768;

// True when `stream` is capturing (or its state cannot be read).
bool stream_capturing(void* stream);

// sorted[i] = points[order[i]] with order by Morton key (0.25-bohr grid);
// stream-ordered, temporary buffers from the stream's pool.  n < 2^31.
int sort_points(const double* points, int64_t n, double* sorted, uint32_t* order, void* stream);

// out[order[i]] = v[i].
int scatter_values(const double* v, const uint32_t* order, int64_t n, double* out, void* stream);

// One instance of a multi-instance scatter: out[order[i]] = v[i], i < n.
struct ScatterDesc {
    const double* v;
    const uint32_t* order;
    double* out;
    int64_t n;
};

// The scatters of n_desc instances in one launch (grid.y = instance).
int scatter_values_multi(const ScatterDesc* d, int n_desc, int64_t max_n, void* stream);

// Rows of 4: out[4 order[i] + c] = v[4 i + c].
int scatter_rows4(const double* v, const uint32_t* order, int64_t n, double* out, void* stream);

}  // namespace envpot
