// The autotuner's cache file for batched circuits (host code only, no
// device calls): one record per (device architecture, qubit count) of
// complex64 batches, read and merged into a small JSON file.
#ifndef SV_TUNE_CACHE_H
#define SV_TUNE_CACHE_H

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <string>
#include <thread>
#include <utility>

#include <unistd.h>

namespace sv {
namespace tunecache {

constexpr int kMaxQubits = 30;  // batch circuits
constexpr int kMaxWidth = 5;    // fusion width
constexpr int kMaxTilesPerWg = 8;

// Tuned figures of one (architecture, qubit count); -1: not tuned.
struct TuneRecord {
    int kmax = -1;
    double persistent_ms = -1.0;  // per circuit, at kmax
    int tiles_per_wg = -1;
    int spread = -1;
    double level_ms = -1.0;  // per circuit, in that shape
};

using Records = std::map<std::pair<std::string, int>, TuneRecord>;  // (arch, n)

// The value of "key" in a one-line JSON object: a string (without quotes)
// or a number, as text; empty if absent.
inline std::string json_field(const std::string& line, const char* key)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = line.find(k);
    if (p == std::string::npos) return {};
    p = line.find(':', p + k.size());
    if (p == std::string::npos) return {};
    ++p;
    while (p < line.size() && line[p] == ' ') ++p;
    if (p < line.size() && line[p] == '"') {
        const size_t e = line.find('"', p + 1);
        return e == std::string::npos ? std::string() : line.substr(p + 1, e - p - 1);
    }
    size_t e = p;
    while (e < line.size() && line[e] != ',' && line[e] != '}' && line[e] != ' ') ++e;
    return line.substr(p, e - p);
}

inline bool json_int(const std::string& v, int lo, int hi, int* out)
{
    if (v.empty()) return false;
    char* end = nullptr;
    const long x = std::strtol(v.c_str(), &end, 10);
    if (*end != '\0' || x < lo || x > hi) return false;
    *out = int(x);
    return true;
}

inline bool json_double(const std::string& v, double* out)
{
    if (v.empty()) return false;
    char* end = nullptr;
    const double x = std::strtod(v.c_str(), &end);
    if (*end != '\0' || !std::isfinite(x)) return false;
    *out = x;
    return true;
}

// Cache file format: {"sv_autotune": 1, "entries": [ one object per line ]},
// each object {"arch": .., "dtype": "c64", "n": .., "kmax": .., "persistent_ms": ..,
// "tiles_per_wg": .., "spread": .., "level_ms": ..}.  Lines that do not parse
// as such an entry are skipped.
inline Records read_tune_file(const std::string& path)
{
    Records out;
    std::FILE* f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    std::string line;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
        line += buf;
        if (line.empty() || line.back() != '\n') continue;  // a line longer than the buffer
        if (json_field(line, "dtype") == "c64") {
            const std::string arch = json_field(line, "arch");
            int n = 0;
            TuneRecord r;
            bool ok = !arch.empty() && json_int(json_field(line, "n"), 1, kMaxQubits, &n);
            ok = ok && json_int(json_field(line, "kmax"), -1, kMaxWidth, &r.kmax);
            ok = ok && json_double(json_field(line, "persistent_ms"), &r.persistent_ms);
            ok = ok && json_int(json_field(line, "tiles_per_wg"), -1, kMaxTilesPerWg, &r.tiles_per_wg);
            ok = ok && json_int(json_field(line, "spread"), -1, 1, &r.spread);
            ok = ok && json_double(json_field(line, "level_ms"), &r.level_ms);
            ok = ok && (r.kmax == -1 || r.kmax >= 1);
            ok = ok && (r.tiles_per_wg == -1 || (r.tiles_per_wg >= 1 && (r.tiles_per_wg & (r.tiles_per_wg - 1)) == 0));
            ok = ok && ((r.tiles_per_wg == -1) == (r.spread == -1));
            if (ok) out[{arch, n}] = r;
        }
        line.clear();
    }
    std::fclose(f);
    return out;
}

// Merges recs into the cache file (entries already there for other keys are
// kept; a key present in both takes recs' figures where recs has them).
// Written to a temporary file and renamed over the old one.  Failures to
// write leave the file as it was and are not errors of the batch.
inline void write_tune_file(const std::string& path, const Records& recs)
{
    auto all = read_tune_file(path);
    for (const auto& kv : recs) {
        TuneRecord& d = all[kv.first];
        const TuneRecord& r = kv.second;
        if (r.kmax != -1) {
            d.kmax = r.kmax;
            d.persistent_ms = r.persistent_ms;
        }
        if (r.tiles_per_wg != -1) {
            d.tiles_per_wg = r.tiles_per_wg;
            d.spread = r.spread;
            d.level_ms = r.level_ms;
        }
    }
    const std::string tmp = path + ".tmp." + std::to_string(long(getpid())) + "." +
                            std::to_string(uint64_t(std::hash<std::thread::id>()(std::this_thread::get_id())));
    std::FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    bool ok = std::fprintf(f, "{\"sv_autotune\": 1, \"entries\": [\n") > 0;
    size_t i = 0;
    for (const auto& kv : all) {
        const TuneRecord& r = kv.second;
        ok = ok && std::fprintf(f,
                                "{\"arch\": \"%s\", \"dtype\": \"c64\", \"n\": %d, \"kmax\": %d, \"persistent_ms\": %.6g, "
                                "\"tiles_per_wg\": %d, \"spread\": %d, \"level_ms\": %.6g}%s\n",
                                kv.first.first.c_str(), kv.first.second, r.kmax, r.persistent_ms, r.tiles_per_wg,
                                r.spread, r.level_ms, ++i < all.size() ? "," : "") > 0;
    }
    ok = ok && std::fprintf(f, "]}\n") > 0;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}


}  // namespace tunecache
}  // namespace sv

#endif
