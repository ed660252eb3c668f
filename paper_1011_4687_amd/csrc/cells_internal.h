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

// Mailbox of the resident single-point mode, in pinned fine-grained host
// memory: the host posts a position and its sequence number, the kernel
// answers with V and the same number.  Written by the host: point,
// req_seq, stop; by the kernel: value, done_seq, running (0 at its exit).
struct CellMailbox {
    double point[3];
    uint64_t req_seq;
    double value;
    uint64_t done_seq;
    uint32_t stop;
    uint32_t running;
};

// Device memory: workgroup 0 relays each position (cmd 1) or the exit
// (cmd 0) to the other workgroups.
struct CellRelay {
    double point[3];
    uint64_t seq;
    uint32_t cmd;
    uint32_t pad;
};

struct CellResidentArgs {
    CellMailbox* box;
    CellRelay* relay;        // seq = start_seq, cmd = 0 at launch
    const uint32_t* cells;
    int64_t m;
    const double* nuc;
    int32_t n_nuc;
    int32_t pad;
    double* part;            // one partial per workgroup
    unsigned int* ticket;    // 0 at launch
    uint64_t start_seq;      // the mailbox's done_seq at launch
    uint64_t idle_ticks;     // real-time-counter ticks without a position before exiting
    uint64_t grace_ticks;    // extra ticks the other workgroups wait for workgroup 0's relay
};

int launch_cells(const CellArgs& a, int S, int precision, int np, void* stream);
int launch_cells_one(const CellOneArgs& a, int grid, int precision, void* stream);
int launch_cells_resident(const CellResidentArgs& a, int grid, int precision, void* stream);

}  // namespace envpot
