// Host-side check of the tile sweeps' geometry: builds the tile arguments
// with the library's own make_tile_args and replays, on the CPU, the index
// arithmetic the tile kernels perform with them (tile base, run offsets,
// group bases, per-matrix-index LDS offsets).  Checks, for every layout
// (plain, spread, strided) and kernel shape, that the tiles cover every
// amplitude exactly once, that each group's 2^k members differ from its
// base exactly by the target bits of their matrix index, and that the run
// boundary keeps a wave's vectors in one run.  Exit status 0 = all passed.
#include "../paper_2308_01999_amd/csrc/sv_apply.hip"

#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

using namespace sv;

static uint64_t h_insert(uint64_t v, const int32_t* pos, int n)
{
    for (int j = 0; j < n; ++j) {
        const int p = pos[j];
        const uint64_t lo = v & ((uint64_t(1) << p) - 1);
        v = ((v >> p) << (p + 1)) | lo;
    }
    return v;
}

static uint64_t h_deposit(uint64_t r, const int32_t* pos, int n)
{
    uint64_t o = 0;
    for (int b = 0; b < n; ++b) o |= ((r >> b) & 1u) << pos[b];
    return o;
}

static uint64_t h_tile_base(uint64_t t, const TileArgs& a)
{
    if (a.trot > 0) t = ((t & ((uint64_t(1) << a.trot) - 1)) << (a.lg_tiles - a.trot)) | (t >> a.trot);
    return h_insert(t << a.L, a.hi_pos, a.n_hi);
}

static int fails = 0;
static int spread_used = 0, strided_used = 0;

static void fail(const char* what, int n, int tb, const std::vector<int>& tg, int spread, bool strided)
{
    if (++fails <= 10) {
        printf("FAIL %s: n=%d tb=%d spread=%d strided=%d targets", what, n, tb, spread, int(strided));
        for (int q : tg) printf(" %d", q);
        printf("\n");
    }
}

// min_L: smallest run width the kernel's wave layout allows (7 when a
// 64-lane wave covers 128 complex64 amplitudes, 6 for 64 complex128).
static void check(int n, int tb, int min_L, const std::vector<int>& tg, int spread, bool strided, int cu)
{
    GateDesc d{};
    d.n = n;
    d.k = int(tg.size());
    for (int a = 0; a < d.k; ++a) d.tbit[a] = uint64_t(1) << tg[a];
    const TileArgs t = make_tile_args(d, n, tb, cu, spread, strided);
    if (t.L < min_L) return fail("run shorter than a wave", n, tb, tg, spread, strided);
    if (t.L + t.n_hi != tb || t.n_lo != d.k || t.n_hi > SV_MAX_TARGETS)
        return fail("tile bit counts", n, tb, tg, spread, strided);
    for (int j = 1; j < t.n_lo; ++j)
        if (t.lo_pos[j] <= t.lo_pos[j - 1]) return fail("lo_pos order", n, tb, tg, spread, strided);
    for (int j = 0; j < t.n_hi; ++j)
        if (t.hi_pos[j] < t.L || t.hi_pos[j] >= n || (j && t.hi_pos[j] <= t.hi_pos[j - 1]))
            return fail("hi_pos", n, tb, tg, spread, strided);
    if (t.n_tiles != (uint64_t(1) << (n - tb)) || t.tiles_per_wg < 1) return fail("tile count", n, tb, tg, spread, strided);
    spread_used += t.L < tb - d.k + 1 && t.n_hi > 0 && [&] {
        for (int j = 0; j < t.n_hi; ++j) {
            bool is_t = false;
            for (int q : tg) is_t |= q == t.hi_pos[j];
            if (!is_t) return true;
        }
        return false;
    }();
    strided_used += t.trot > 0;
    const uint64_t N = uint64_t(1) << n;
    const uint64_t T = uint64_t(1) << tb;
    const uint64_t mask = (uint64_t(1) << t.L) - 1;
    uint64_t tbits = 0;
    for (int a = 0; a < d.k; ++a) tbits |= d.tbit[a];
    std::vector<uint8_t> seen(N, 0), lseen(T);
    for (uint64_t tile = 0; tile < t.n_tiles; ++tile) {
        const uint64_t base = h_tile_base(tile, t);
        auto glob = [&](uint64_t i) { return base + h_deposit(i >> t.L, t.hi_pos, t.n_hi) + (i & mask); };
        for (uint64_t i = 0; i < T; ++i) {
            const uint64_t gi = glob(i);
            if (gi >= N || seen[gi]) return fail("tile coverage", n, tb, tg, spread, strided);
            seen[gi] = 1;
        }
        std::fill(lseen.begin(), lseen.end(), 0);
        for (uint64_t g = 0; g < (T >> d.k); ++g) {
            const uint64_t pb = h_insert(g, t.lo_pos, t.n_lo);
            if (pb >= T) return fail("group base outside the tile", n, tb, tg, spread, strided);
            const uint64_t g0 = glob(pb);
            if (g0 & tbits) return fail("group base has target bits", n, tb, tg, spread, strided);
            for (int c = 0; c < (1 << d.k); ++c) {
                const uint64_t li = pb + uint64_t(t.lds_off[c]);
                uint64_t want = g0;
                for (int a = 0; a < d.k; ++a)
                    if ((c >> a) & 1) want |= d.tbit[a];
                if (li >= T || lseen[li] || glob(li) != want) return fail("group member", n, tb, tg, spread, strided);
                lseen[li] = 1;
            }
        }
    }
}

// The same checks on a sample of the tiles, for states too large to
// enumerate (up to 34 qubits): the first, the last and 62 random tiles; the
// amplitudes of distinct sampled tiles must all differ and lie below 2^n.
static void check_sampled(int n, int tb, int min_L, const std::vector<int>& tg, int spread, bool strided, int cu,
                          std::mt19937_64& rng)
{
    GateDesc d{};
    d.n = n;
    d.k = int(tg.size());
    for (int a = 0; a < d.k; ++a) d.tbit[a] = uint64_t(1) << tg[a];
    const TileArgs t = make_tile_args(d, n, tb, cu, spread, strided);
    if (t.L < min_L) return fail("run shorter than a wave (sampled)", n, tb, tg, spread, strided);
    if (t.L + t.n_hi != tb || t.n_lo != d.k) return fail("tile bit counts (sampled)", n, tb, tg, spread, strided);
    if (t.n_tiles != (uint64_t(1) << (n - tb))) return fail("tile count (sampled)", n, tb, tg, spread, strided);
    strided_used += t.trot > 0;
    const uint64_t N = uint64_t(1) << n;
    const uint64_t T = uint64_t(1) << tb;
    const uint64_t mask = (uint64_t(1) << t.L) - 1;
    uint64_t tbits = 0;
    for (int a = 0; a < d.k; ++a) tbits |= d.tbit[a];
    std::vector<uint64_t> tiles = {0, t.n_tiles - 1};
    for (int r = 0; r < 62; ++r) tiles.push_back(rng() % t.n_tiles);
    std::sort(tiles.begin(), tiles.end());
    tiles.erase(std::unique(tiles.begin(), tiles.end()), tiles.end());
    std::vector<uint64_t> all;
    all.reserve(tiles.size() * T);
    std::vector<uint8_t> lseen(T);
    for (uint64_t tile : tiles) {
        const uint64_t base = h_tile_base(tile, t);
        auto glob = [&](uint64_t i) { return base + h_deposit(i >> t.L, t.hi_pos, t.n_hi) + (i & mask); };
        for (uint64_t i = 0; i < T; ++i) {
            const uint64_t gi = glob(i);
            if (gi >= N) return fail("tile coverage (sampled)", n, tb, tg, spread, strided);
            all.push_back(gi);
        }
        std::fill(lseen.begin(), lseen.end(), 0);
        for (uint64_t g = 0; g < (T >> d.k); ++g) {
            const uint64_t pb = h_insert(g, t.lo_pos, t.n_lo);
            const uint64_t g0 = glob(pb);
            if (pb >= T || (g0 & tbits)) return fail("group base (sampled)", n, tb, tg, spread, strided);
            for (int c = 0; c < (1 << d.k); ++c) {
                const uint64_t li = pb + uint64_t(t.lds_off[c]);
                uint64_t want = g0;
                for (int a = 0; a < d.k; ++a)
                    if ((c >> a) & 1) want |= d.tbit[a];
                if (li >= T || lseen[li] || glob(li) != want) return fail("group member (sampled)", n, tb, tg, spread, strided);
                lseen[li] = 1;
            }
        }
    }
    std::sort(all.begin(), all.end());
    if (std::adjacent_find(all.begin(), all.end()) != all.end())
        return fail("tiles overlap (sampled)", n, tb, tg, spread, strided);
}

int main()
{
    // (tile bits, targets, min run width) of every tile kernel
    struct Shape {
        int tb, k, min_L;
    };
    const Shape shapes[] = {{12, 4, 7}, {12, 5, 7}, {13, 5, 7}, {11, 5, 6}, {12, 5, 6}, {13, 6, 7}, {12, 6, 6},
                            // the permutation-gate tiles (per-lane addresses: any run width)
                            {12, 1, 0}, {12, 2, 0}, {12, 3, 0}, {12, 6, 0}, {11, 1, 0}, {11, 3, 0}, {11, 6, 0}};
    std::mt19937 rng(7);
    int cases = 0;
    for (const Shape& sh : shapes)
        for (int n = sh.tb; n <= sh.tb + 7; ++n)
            for (int layout = 0; layout < 4; ++layout) {
                const int spread = (layout & 1) ? 12 : 0;
                const bool strided = (layout & 2) != 0;
                for (int rep = 0; rep < (n > sh.tb + 5 ? 6 : 14); ++rep) {
                    std::vector<int> tg(sh.k);
                    if (rep <= n - sh.k && rep < 8) {
                        for (int a = 0; a < sh.k; ++a) tg[a] = rep + a;  // windows of adjacent qubits
                    } else {
                        std::vector<int> q(n);
                        for (int i = 0; i < n; ++i) q[i] = i;
                        std::shuffle(q.begin(), q.end(), rng);
                        std::copy(q.begin(), q.begin() + sh.k, tg.begin());
                    }
                    // 1 CU: many tiles per workgroup, so the strided order is exercised
                    check(n, sh.tb, sh.min_L, tg, spread, strided, (rep & 1) ? 1 : 256);
                    ++cases;
                }
            }
    // large states, sampled tiles: targets anywhere up to the top qubit
    std::mt19937_64 rng64(11);
    int sampled = 0;
    for (const Shape& sh : shapes)
        for (int n : {sh.tb + 8, 24, 28, 31, 33, 34}) {
            if (n <= sh.tb + 7) continue;
            for (int layout = 0; layout < 4; ++layout) {
                const int spread = (layout & 1) ? 12 : 0;
                const bool strided = (layout & 2) != 0;
                for (int rep = 0; rep < 3; ++rep) {
                    std::vector<int> q(n);
                    for (int i = 0; i < n; ++i) q[i] = i;
                    std::shuffle(q.begin(), q.end(), rng);
                    std::vector<int> tg(q.begin(), q.begin() + sh.k);
                    if (rep == 0) tg[0] = n - 1;  // the top qubit
                    std::sort(tg.begin(), tg.end());
                    tg.erase(std::unique(tg.begin(), tg.end()), tg.end());
                    if (int(tg.size()) != sh.k) continue;
                    check_sampled(n, sh.tb, sh.min_L, tg, spread, strided, (rep & 1) ? 1 : 256, rng64);
                    ++sampled;
                }
            }
        }
    printf("cases %d sampled %d fails %d spread-layout %d strided %d\n", cases, sampled, fails, spread_used,
           strided_used);
    return (fails == 0 && spread_used > 0 && strided_used > 0) ? 0 : 1;
}
