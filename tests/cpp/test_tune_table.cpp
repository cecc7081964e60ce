// Host check of the tuner's text records (tune_table.h): well-formed lines in both forms,
// blank lines, and a list of malformed ones; then random records written and read back.
#include "tune_table.h"

#include <cstdio>
#include <cstring>
#include <random>
#include <string>

static bool width_ok(int tw) { return tw == 8 || tw == 16 || tw == 32 || tw == 64; }

static int fails = 0;
static void expect(const char* line, int want) {
    qc::TuneKey k;
    qc::TuneEntry e;
    const int got = qc::parse_tune_line(line, &k, &e, width_ok);
    if (got != want) {
        std::printf("line \"%s\": got %d, want %d\n", line, got, want);
        ++fails;
    }
}

int main() {
    // well-formed
    expect("640 480 7 5 1 0 16 0\n", 1);
    expect("640 480 7 5 1 0 32 2", 1);
    expect("  512\t424 18 3 3 1 8 2 \r\n", 1);
    expect("640 480 7 5 16\n", 1);            // older five-field form
    expect("\n", 0);
    expect("   \t \r\n", 0);
    expect("", 0);
    // malformed
    const char* bad[] = {
        "640 480 7 5 1 0 16\n",             // seven fields
        "640 480 7 5 1 0 16 0 9\n",         // nine fields
        "640 480 7\n",                      // three fields
        "640 480 7 5 1 0 16 1\n",           // schedule FP32 is not a tuned schedule
        "640 480 7 5 1 0 24 0\n",           // tile width 24
        "640 480 0 5 1 0 16 0\n",           // radius 0
        "640 480 19 5 1 0 16 0\n",          // radius beyond QC_MAX_RADIUS
        "640 480 7 -1 1 0 16 0\n",          // negative iterations
        "640 480 7 5 8 0 16 0\n",           // stride beyond the radius
        "640 480 7 5 0 0 16 0\n",           // stride 0
        "640 480 7 5 1 2 16 0\n",           // reject not 0/1
        "0 480 7 5 1 0 16 0\n",             // width 0
        "640 480 7 5 1 0 16 0x\n",          // junk glued to a number
        "640 480 7.5 5 1 0 16 0\n",         // not an integer
        "# 640 480 7 5 1 0 16 0\n",         // comments are not part of the format
        "640 480 7 5 1 0 16 99999999999999999999\n",   // beyond long
        "640 480 7 5 1 0 16 4294967296\n",  // beyond int
        "640 480 7 5 1 0 16 -\n",           // a sign alone
    };
    for (const char* b : bad) expect(b, -1);

    // round trip of random valid records through the writer
    std::mt19937 rng(1707);
    const int widths[4] = {8, 16, 32, 64};
    for (int i = 0; i < 20000; ++i) {
        const int r = 1 + int(rng() % QC_MAX_RADIUS);
        const qc::TuneKey k{1 + int(rng() % 8192), 1 + int(rng() % 8192), r, int(rng() % 50),
                            1 + int(rng() % r), int(rng() % 2)};
        qc::TuneEntry e;
        e.tile_width = widths[rng() % 4];
        e.schedule = rng() % 2 ? QC_PREC_FP64 : QC_PREC_MIXED;
        char buf[256];
        std::FILE* f = fmemopen(buf, sizeof buf, "w");
        qc::format_tune_line(f, k, e);
        std::fclose(f);
        qc::TuneKey k2;
        qc::TuneEntry e2;
        if (qc::parse_tune_line(buf, &k2, &e2, width_ok) != 1 || k2 != k || e2.tile_width != e.tile_width ||
            e2.schedule != e.schedule) {
            std::printf("round trip failed: %s", buf);
            ++fails;
            break;
        }
    }
    std::printf(fails ? "FAIL\n" : "OK\n");
    return fails ? 1 : 0;
}
