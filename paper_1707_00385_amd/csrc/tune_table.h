// tune_table.h -- the tuner's records and their text form (host-side only).
//
// One record per line: "width height radius iterations stride reject tile_width schedule"
// (eight decimal integers), or the older "width height radius iterations tile_width"
// (stride 1, no rejection, schedule MIXED).  Blank lines are skipped; anything else is
// malformed.
#pragma once

#include <cerrno>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <tuple>

#include "qcurv.h"

namespace qc {

// width, height, radius, iterations, stride, reject
using TuneKey = std::tuple<int, int, int, int, int, int>;

// What qc_tune recorded for a key: the FP32 pass's tile width, and the schedule of a MIXED
// request: QC_PREC_MIXED (the FP32 pass plus the FP64 recomputation of listed pixels) or
// QC_PREC_FP64 (every pixel in FP64, where that measured faster).
struct TuneEntry {
    int tile_width = 16;
    int schedule = QC_PREC_MIXED;
};

// Parses one line.  Returns 0 for a blank line, 1 for a valid record (stored in *key and
// *entry), -1 for anything else: a field that is not a decimal integer in int range,
// a field count other than 5 or 8, or a value outside what qc_fit accepts
// (tile_width_ok decides the tile width).
inline int parse_tune_line(const char* line, TuneKey* key, TuneEntry* entry, bool (*tile_width_ok)(int)) {
    long v[8];
    int n = 0;
    const char* p = line;
    for (;;) {
        while (*p == ' ' || *p == '\t' || *p == '\r' || *p == '\n') ++p;
        if (*p == '\0') break;
        if (n == 8) return -1;
        char* end = nullptr;
        errno = 0;
        const long x = std::strtol(p, &end, 10);
        if (end == p || errno == ERANGE || x < INT_MIN || x > INT_MAX) return -1;
        if (*end != '\0' && *end != ' ' && *end != '\t' && *end != '\r' && *end != '\n') return -1;
        v[n++] = x;
        p = end;
    }
    if (n == 0) return 0;
    int w, h, r, t, stride = 1, reject = 0, tw, sched = QC_PREC_MIXED;
    if (n == 5) {
        w = int(v[0]); h = int(v[1]); r = int(v[2]); t = int(v[3]); tw = int(v[4]);
    } else if (n == 8) {
        w = int(v[0]); h = int(v[1]); r = int(v[2]); t = int(v[3]);
        stride = int(v[4]); reject = int(v[5]); tw = int(v[6]); sched = int(v[7]);
    } else {
        return -1;
    }
    if (w < 1 || h < 1 || r < 1 || r > QC_MAX_RADIUS || t < 0 || stride < 1 || stride > r ||
        (reject != 0 && reject != 1) || !tile_width_ok(tw) ||
        (sched != QC_PREC_MIXED && sched != QC_PREC_FP64))
        return -1;
    *key = TuneKey{w, h, r, t, stride, reject};
    entry->tile_width = tw;
    entry->schedule = sched;
    return 1;
}

// Writes one record as parse_tune_line reads it (eight fields).
inline int format_tune_line(std::FILE* f, const TuneKey& k, const TuneEntry& e) {
    return std::fprintf(f, "%d %d %d %d %d %d %d %d\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                        std::get<3>(k), std::get<4>(k), std::get<5>(k), e.tile_width, e.schedule);
}

}  // namespace qc
