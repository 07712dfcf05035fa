// Host check of the batched autotuner's cache file (no GPU needed): records
// written and read back, merging by key, partial records, and lines that
// must be skipped (out-of-range or missing fields, other state types,
// garbage).  Usage: tune_cache_check <scratch directory>.  Prints "fails N".
#include "../paper_2308_01999_amd/csrc/sv_tune_cache.h"

#include <cstdio>
#include <string>

using namespace sv::tunecache;

static int fails = 0;

static void check(bool ok, const char* what)
{
    if (!ok) {
        ++fails;
        std::printf("FAIL %s\n", what);
    }
}

static TuneRecord rec(int kmax, double pm, int tpw, int spread, double lm)
{
    TuneRecord r;
    r.kmax = kmax;
    r.persistent_ms = pm;
    r.tiles_per_wg = tpw;
    r.spread = spread;
    r.level_ms = lm;
    return r;
}

static bool same(const TuneRecord& a, const TuneRecord& b)
{
    return a.kmax == b.kmax && a.tiles_per_wg == b.tiles_per_wg && a.spread == b.spread &&
           std::fabs(a.persistent_ms - b.persistent_ms) <= 1e-6 * std::fabs(b.persistent_ms) + 1e-12 &&
           std::fabs(a.level_ms - b.level_ms) <= 1e-6 * std::fabs(b.level_ms) + 1e-12;
}

int main(int argc, char** argv)
{
    if (argc < 2) return 2;
    const std::string dir = argv[1];
    const std::string path = dir + "/tune.json";
    std::remove(path.c_str());

    // a missing file reads as empty
    check(read_tune_file(path).empty(), "missing file is empty");

    // round trip
    Records a;
    a[{"gfx950:sramecc+:xnack-", 10}] = rec(4, 0.0123, -1, -1, -1.0);
    a[{"gfx950:sramecc+:xnack-", 15}] = rec(5, 0.25, 2, 0, 0.2);
    a[{"gfx942", 20}] = rec(-1, -1.0, 8, 1, 3.5);
    write_tune_file(path, a);
    Records b = read_tune_file(path);
    check(b.size() == 3, "three records read back");
    for (const auto& kv : a) check(b.count(kv.first) && same(b[kv.first], kv.second), "record read back unchanged");

    // merging: a new key is added, a partial record keeps the other part
    write_tune_file(path, {{{"gfx950:sramecc+:xnack-", 12}, rec(3, 0.01, -1, -1, -1.0)}});
    write_tune_file(path, {{{"gfx942", 20}, rec(4, 1.5, -1, -1, -1.0)}});
    b = read_tune_file(path);
    check(b.size() == 4, "four records after merging");
    check(same(b[{"gfx942", 20}], rec(4, 1.5, 8, 1, 3.5)), "partial record merged into the existing one");
    check(same(b[{"gfx950:sramecc+:xnack-", 15}], rec(5, 0.25, 2, 0, 0.2)), "other record kept");

    // lines that must be skipped
    {
        std::FILE* f = std::fopen(path.c_str(), "w");
        std::fprintf(f, "{\"sv_autotune\": 1, \"entries\": [\n");
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 9, \"kmax\": 4, \"persistent_ms\": 0.5, "
                        "\"tiles_per_wg\": -1, \"spread\": -1, \"level_ms\": -1},\n");
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 11, \"kmax\": 9, \"persistent_ms\": 0.5, "
                        "\"tiles_per_wg\": -1, \"spread\": -1, \"level_ms\": -1},\n");  // width out of range
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 17, \"kmax\": -1, \"persistent_ms\": -1, "
                        "\"tiles_per_wg\": 3, \"spread\": 1, \"level_ms\": 2},\n");  // not a power of two
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 18, \"kmax\": -1, \"persistent_ms\": -1, "
                        "\"tiles_per_wg\": 4, \"spread\": -1, \"level_ms\": 2},\n");  // shape half missing
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 31, \"kmax\": 5, \"persistent_ms\": 1, "
                        "\"tiles_per_wg\": -1, \"spread\": -1, \"level_ms\": -1},\n");  // too many qubits
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c128\", \"n\": 12, \"kmax\": 5, \"persistent_ms\": 1, "
                        "\"tiles_per_wg\": -1, \"spread\": -1, \"level_ms\": -1},\n");  // other state type
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 13, \"kmax\": 5, "
                        "\"tiles_per_wg\": -1, \"spread\": -1, \"level_ms\": -1},\n");  // a field missing
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 14, \"kmax\": 5x, \"persistent_ms\": 1, "
                        "\"tiles_per_wg\": -1, \"spread\": -1, \"level_ms\": -1},\n");  // not a number
        std::fprintf(f, "garbage line\n");
        std::fprintf(f, "{\"arch\": \"gfx950\", \"dtype\": \"c64\", \"n\": 16, \"kmax\": 3, \"persistent_ms\": 0.75, "
                        "\"tiles_per_wg\": 1, \"spread\": 0, \"level_ms\": 0.5}\n");
        std::fprintf(f, "]}\n");
        std::fclose(f);
    }
    b = read_tune_file(path);
    check(b.size() == 2, "only the two well-formed records read");
    check(b.count({"gfx950", 9}) && same(b[{"gfx950", 9}], rec(4, 0.5, -1, -1, -1.0)), "record n=9");
    check(b.count({"gfx950", 16}) && same(b[{"gfx950", 16}], rec(3, 0.75, 1, 0, 0.5)), "record n=16");

    // a file that cannot be written leaves nothing behind and is no error
    const std::string bad = dir + "/no_such_dir/tune.json";
    write_tune_file(bad, a);
    check(read_tune_file(bad).empty(), "unwritable path stays empty");

    // leave the round-trip file for the caller to parse as JSON
    std::remove(path.c_str());
    write_tune_file(path, a);
    std::printf("fails %d\n", fails);
    return fails == 0 ? 0 : 1;
}
