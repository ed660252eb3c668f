// Internal layout of the field evaluation E = -grad V (one order of the
// Hermite recursion more than the potential).  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "envpot_internal.h"

namespace envpot {

// Boys tables of the field: F_0 .. F_{L+1} for L <= 4 with the Taylor steps
// of the potential's tables, so more columns, and far-field thresholds from
// F_0 .. F_{L+1} (the asymptote must hold one order higher).
constexpr int kFieldRowF32 = 12;   // floats per row: F_0..F_11 (F_10 is the highest used)
constexpr int kFieldRowF64 = 16;   // doubles per row: F_0..F_15 (F_14 is the highest used)
constexpr int kFieldMaxRowsF32 = 8 * 40 + 1;

struct FieldParams {
    // squared far-field radius of the field for a pair of angular momentum L:
    // the pair record's r2far (= tfar[L]/p) times ratio[L] (= tfarfield[L]/tfar[L])
    float ratio32[kLMax + 1];
    float cl_ratio32;              // the largest ratio, for same-centre clusters
    double ratio64[kLMax + 1];
    double cl_ratio64;
    int32_t rows32;                // rows of the FP32 table (staged into LDS)
    int32_t rows64;
};

struct FieldArgs {
    const double* pts;       // n x 3
    int64_t n;
    const Segment* segs;     // segments of the chosen split factor
    const int32_t* split;    // S+1 offsets into segs
    const uint32_t* rec;     // pair and cluster records of the handle's precision
    const double* nuc;       // nuclei, 4 doubles each
    const void* boys;        // field Boys table of the handle's precision
    const double* boxes;     // segment boxes (Segment::box), or nullptr: test every pair
    double* out;             // S == 1: [n][4] (V, Ex, Ey, Ez); S > 1: partials [S][n][4]
    FieldParams fp;
};

// Host tables and thresholds (both precisions; bp holds the potential's thresholds).
void build_field_tables(const BoysParams& bp, std::vector<float>& t32, std::vector<double>& t64,
                        FieldParams& fp);

// Boys helpers of the pair-list builder (long double).
void boys_ld(int nmax, long double T, long double* F);
double far_threshold(int L, long double eps);

int launch_field(const FieldArgs& a, int S, int precision, int np, void* stream);

}  // namespace envpot
