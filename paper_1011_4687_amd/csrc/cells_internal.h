// Internal layout of the cell-sum environment (the paper's own form of the
// environment: nuclei plus point-charge cells).  Not part of the C ABI.
#pragma once

#include <cstdint>

namespace envpot {

// One cell record, 8 words: x, y, z (FP64) and the cell's electron count q,
// FP64 for the FP64 path, FP32 (plus a pad word) for the FP32C path.
constexpr int kCellWords = 8;
constexpr int kCellTile = 16;       // cells per FP32 partial sum (FP32C)
constexpr int kCellsPaperGrid = 120;  // the paper's launch: 120 blocks x 256 threads

struct CellArgs {
    const double* pts;       // n x 3
    int64_t n;
    const uint32_t* cells;   // records
    const int32_t* split;    // S + 1 cell offsets
    const double* nuc;       // K x 4 (x, y, z, Z)
    int32_t n_nuc;
    int32_t pad;
    double* out;             // S == 1: V; S > 1: partials [S][n]
};

struct CellOneArgs {
    const double* pt;        // one point (3 doubles, device)
    const uint32_t* cells;
    int64_t m;               // cells
    const double* nuc;
    int32_t n_nuc;
    int32_t pad;
    double* part;            // one partial per workgroup
    unsigned int* ticket;    // workgroups finished (reset by the last one)
    double* out;             // V at the point
};

int launch_cells(const CellArgs& a, int S, int precision, int np, void* stream);
int launch_cells_one(const CellOneArgs& a, int grid, int precision, void* stream);

}  // namespace envpot
