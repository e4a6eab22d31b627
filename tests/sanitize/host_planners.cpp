// Host-side planners of the HIP library under AddressSanitizer and
// UndefinedBehaviorSanitizer (host code only; no GPU call is made): the
// workspace plan, the workgroup blocking of the gather layout, the link and
// stream blocking and the host-built tile tables of the binned layout, and
// the batched layout's tiling and host validation, on ragged patterns (empty
// rows and routes, rows longer than one workgroup's stage, single rows).
// The translation unit includes the two sources whose helpers have internal
// linkage; the other sources are linked as usual.
#include "pmp_api.hip"
#include "pmp_batch.hip"

#include <cstdio>
#include <cstdlib>
#include <random>

#define REQUIRE(cond)                                                          \
    do {                                                                       \
        if (!(cond)) {                                                         \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            std::exit(1);                                                      \
        }                                                                      \
    } while (0)

struct Csr {
    int m = 0, n = 0;
    std::vector<int> row_ptr, col_idx;
};

// Random pattern with distinct columns per row; `deg_hi` bounds the row
// length, `heavy` rows get `heavy_len` entries, a fraction of rows is empty.
static Csr random_csr(std::mt19937 &g, int m, int n, int deg_hi, int heavy, int heavy_len)
{
    Csr a;
    a.m = m;
    a.n = n;
    a.row_ptr.assign((size_t)m + 1, 0);
    std::vector<char> used((size_t)n, 0);
    for (int l = 0; l < m; ++l) {
        int d = (g() % 5 == 0) ? 0 : (int)(g() % (unsigned)(deg_hi + 1));
        if (l < heavy) d = heavy_len;
        d = std::min(d, n);
        std::vector<int> cols;
        while ((int)cols.size() < d) {
            const int j = (int)(g() % (unsigned)n);
            if (!used[(size_t)j]) {
                used[(size_t)j] = 1;
                cols.push_back(j);
            }
        }
        for (int j : cols) used[(size_t)j] = 0;
        std::sort(cols.begin(), cols.end());
        a.col_idx.insert(a.col_idx.end(), cols.begin(), cols.end());
        a.row_ptr[(size_t)l + 1] = (int)a.col_idx.size();
    }
    return a;
}

static std::vector<int> csc_ptr(const Csr &a)
{
    std::vector<int> p((size_t)a.n + 1, 0);
    for (int j : a.col_idx) p[(size_t)j + 1]++;
    for (int j = 0; j < a.n; ++j) p[(size_t)j + 1] += p[(size_t)j];
    return p;
}

static void check_blocks(const std::vector<int> &ptr, int count)
{
    const std::vector<int> b = make_blocks(ptr, count);
    REQUIRE(b.front() == 0 && b.back() == count);
    for (size_t i = 1; i < b.size(); ++i) {
        REQUIRE(b[i] > b[i - 1]);
        const long long nz = (long long)ptr[(size_t)b[i]] - ptr[(size_t)b[i - 1]];
        REQUIRE(b[i] - b[i - 1] <= kBlock);
        REQUIRE(nz <= kCap || b[i] - b[i - 1] == 1);
    }
}

static void check_binned(const Csr &a)
{
    const long long nnz = (long long)a.col_idx.size();
    const BinnedPlan bound = binned_plan(a.m, a.n, nnz);
    std::vector<int> lbs((size_t)bound.P + 1), sbs((size_t)bound.Q + 1);
    BinnedPlan bp = bound;
    binned_blocks(a.row_ptr.data(), a.m, a.n, nnz, bp, lbs.data(), sbs.data());
    REQUIRE(bp.P <= bound.P && bp.Q <= bound.Q && bp.LB <= bound.LB && bp.SB <= bound.SB);
    REQUIRE(bp.LB <= kBinMaxBlock && bp.SB <= kBinMaxBlock);
    REQUIRE(lbs[0] == 0 && lbs[(size_t)bp.P] == a.m && sbs[0] == 0 && sbs[(size_t)bp.Q] == a.n);
    for (int p = 0; p < bp.P; ++p) REQUIRE(lbs[(size_t)p + 1] - lbs[(size_t)p] <= bp.LB);
    const size_t tiles = (size_t)bp.P * bp.Q;
    std::vector<int> ox(tiles + 1), ov(tiles + 1);
    std::vector<uint16_t> lix((size_t)nnz + 4), six((size_t)nnz + 4);
    binned_build_host(a.row_ptr.data(), a.col_idx.data(), a.m, a.n, bp, lbs.data(), sbs.data(),
                      ox.data(), ov.data(), lix.data(), six.data(), 1);
    REQUIRE(ox[0] == 0 && ox[tiles] == nnz && ov[0] == 0 && ov[tiles] == nnz);
    for (size_t t = 0; t < tiles; ++t) REQUIRE(ox[t] <= ox[t + 1] && ov[t] <= ov[t + 1]);
    // every nonzero appears once, at its own link and stream
    std::vector<long long> seen((size_t)a.m, 0);
    for (int p = 0; p < bp.P; ++p)
        for (int q = 0; q < bp.Q; ++q) {
            const size_t tx = (size_t)p * bp.Q + q, tv = (size_t)q * bp.P + p;
            const int len = ox[tx + 1] - ox[tx];
            REQUIRE(len == ov[tv + 1] - ov[tv]);
            for (int k = 0; k < len; ++k) {
                const uint16_t code = lix[(size_t)ox[tx] + k];
                const int l = lbs[(size_t)p] + (code & kLocalMask);
                REQUIRE(((code & kLongBit) != 0) ==
                        (a.row_ptr[(size_t)l + 1] - a.row_ptr[(size_t)l] > kCap));
                const int j = sbs[(size_t)q] + six[(size_t)ov[tv] + k];
                REQUIRE(l < lbs[(size_t)p + 1] && j < sbs[(size_t)q + 1]);
                REQUIRE(std::binary_search(a.col_idx.begin() + a.row_ptr[(size_t)l],
                                           a.col_idx.begin() + a.row_ptr[(size_t)l + 1], j));
                seen[(size_t)l]++;
            }
        }
    for (int l = 0; l < a.m; ++l) REQUIRE(seen[(size_t)l] == a.row_ptr[(size_t)l + 1] - a.row_ptr[(size_t)l]);
}

static pmp_problem host_problem(const Csr &a, std::vector<double> &c, std::vector<double> &w,
                                std::vector<uint8_t> &u, double hi)
{
    pmp_problem p{};
    p.m = a.m;
    p.n = a.n;
    p.nnz = (int64_t)a.col_idx.size();
    p.row_ptr = a.row_ptr.data();
    p.col_idx = a.col_idx.empty() ? nullptr : a.col_idx.data();
    c.assign((size_t)a.m, 2.0);
    w.assign((size_t)a.n, 1.0);
    u.assign((size_t)a.n, 0);
    p.c = c.data();
    p.w = w.data();
    p.utility = u.data();
    p.lo = 0.0;
    p.hi = hi;
    p.dtype = PMP_F64;
    p.memory = PMP_MEM_HOST;
    return p;
}

int main()
{
    std::mt19937 g(1234);
    // workspace plans over edge sizes, both layouts
    const long long shapes[][3] = {{1, 0, 0},   {1, 1, 1},     {7, 3, 5},         {256, 256, 1 << 21},
                                   {300, 70000, 1 << 22}, {5000000, 20000000, 116555391},
                                   {1, 100000, 100000},   {100000, 1, 100000}};
    for (auto &s : shapes)
        for (int layout = 0; layout < 3; ++layout)
            for (size_t sz : {(size_t)4, (size_t)8}) {
                const Layout L = plan((int)s[0], (int)s[1], s[2], sz, layout);
                REQUIRE(L.total > 0 && L.total % 256 == 0);
                REQUIRE(L.nsb_max >= 0 && L.nlb_max >= 0);
            }
    // gather-layout blocking on ragged patterns
    for (int rep = 0; rep < 6; ++rep) {
        const Csr a = random_csr(g, 2000 + 37 * rep, 3000 + 11 * rep, 9, rep, 5000);
        check_blocks(a.row_ptr, a.m);
        check_blocks(csc_ptr(a), a.n);
    }
    {
        std::vector<int> empty(65, 0);
        check_blocks(empty, 64);
        std::vector<int> one = {0, 9000};
        check_blocks(one, 1);
    }
    // binned blocking and tile tables
    const int sizes[][5] = {{700, 900, 6, 0, 0},     {3000, 50000, 12, 2, 20000},
                            {20000, 3000, 4, 3, 2500}, {40000, 120000, 14, 0, 0},
                            {1, 5000, 1, 1, 4000},     {5000, 1, 1, 0, 0}};
    for (auto &z : sizes) check_binned(random_csr(g, z[0], z[1], z[2], z[3], z[4]));
    // batched tiling and host validation
    for (int rep = 0; rep < 4; ++rep) {
        const Csr a = random_csr(g, 800 + rep, 1200 + rep, 7, rep, 4500);
        for (int cap : {64, 1000, 4096}) {
            std::vector<int> seg{0}, owner;
            tiles_for(a.row_ptr, 0, a.m, cap, rep, seg, owner);
            REQUIRE(seg.back() == a.m && owner.size() + 1 == seg.size());
            // link tiles: rows longer than kCap split into chunk tiles that
            // start at their row and cover it once, within the planned bound
            for (int chunk : {1024, 3000, 8192}) {
                std::vector<int> ls{0}, lo;
                std::vector<int2> ck;
                tiles_for(a.row_ptr, 0, a.m, cap, rep, ls, lo, chunk, &ck);
                REQUIRE(ls.back() == a.m && lo.size() + 1 == ls.size() && ck.size() == lo.size());
                BatchSizes z;
                z.M = a.m;
                z.N = a.n;
                z.NNZ = a.row_ptr[(size_t)a.m];
                z.B = 1;
                REQUIRE((long long)lo.size() <= batch_plan(z, 4, cap, chunk).nlt_max);
                for (size_t t = 0; t < lo.size(); ++t) {
                    const int l = ls[t], len = a.row_ptr[(size_t)l + 1] - a.row_ptr[(size_t)l];
                    if (ck[t].y == 0) {
                        REQUIRE(ls[t + 1] > l);
                        continue;
                    }
                    REQUIRE(len > kCap && ck[t].y == (len + chunk - 1) / chunk);
                    REQUIRE(ck[t].x == (t > 0 && ck[t - 1].y > 0 && ls[t - 1] == l ? ck[t - 1].x + 1 : 0));
                    REQUIRE(ls[t + 1] == (ck[t].x + 1 < ck[t].y ? l : l + 1));
                }
            }
        }
        REQUIRE(long_row_shift(8, 5000, 1.0) == 0 && long_row_shift(4, 0, 1.0) == 0);
        REQUIRE(long_row_shift(4, 5000, INFINITY) == 0 && long_row_shift(4, 1LL << 30, 1e9) == 0);
        {
            const int F = long_row_shift(4, 50013, 1e3);
            REQUIRE(F >= 24 && std::ldexp(50013.0 * 1e3, F) <= std::ldexp(1.0, 62) &&
                    std::ldexp(50013.0 * 1e3, F + 1) > std::ldexp(1.0, 62));
        }
        std::vector<double> c, w;
        std::vector<uint8_t> u;
        pmp_problem p = host_problem(a, c, w, u, 10.0);
        REQUIRE(validate_host(p, rep) == PMP_OK);
        size_t bytes = 0;
        pmp_params prm;
        pmp_params_default(&prm);
        REQUIRE(pmp_workspace_size(&p, &prm, &bytes) == PMP_OK && bytes > 0);
        pmp_batch_options opt;
        pmp_batch_options_default(&opt);
        REQUIRE(pmp_batch_workspace_size(1, &p, &prm, &opt, &bytes) == PMP_OK && bytes > 0);
        // each invalid variant is refused without reading out of bounds
        Csr bad = a;
        if (!bad.col_idx.empty()) {
            bad.col_idx[0] = a.n + 5;
            pmp_problem q = host_problem(bad, c, w, u, 10.0);
            REQUIRE(validate_host(q, rep) == PMP_ERR_INVALID);
        }
        c[3] = -1.0;
        REQUIRE(validate_host(p, rep) == PMP_ERR_INVALID);
        c[3] = 2.0;
        w[1] = std::nan("");
        REQUIRE(validate_host(p, rep) == PMP_ERR_INVALID);
        w[1] = 1.0;
        u[2] = 9;
        REQUIRE(validate_host(p, rep) == PMP_ERR_INVALID);
        u[2] = 0;
        Csr wide = a;                 // one more stream, on no route
        wide.n += 1;
        pmp_problem inf = host_problem(wide, c, w, u, INFINITY);
        REQUIRE(validate_host(inf, rep) == PMP_ERR_INVALID);
        inf.hi = 10.0;
        REQUIRE(validate_host(inf, rep) == PMP_OK);
    }
    // the batch kernel's index maps: each phase's tiles dealt to the grid
    // exactly once, and the barrier groups adding up to the grid
    for (unsigned G : {1u, 5u, 8u, 9u, 100u, 512u, 1000u, 1024u}) {
        unsigned total = 0;
        for (unsigned x = 0; x < barrier_groups(G); ++x) total += barrier_group_size(x, G);
        REQUIRE(total == G);
        for (int count : {0, 1, 7, 100, 10711, 24437}) {
            std::vector<int> seen((size_t)count, 0);
            for (unsigned b = 0; b < G; ++b)
                for (TileRange r = xcd_tiles_of(count, G, b); r.t < r.end; r.t += r.step) {
                    REQUIRE(r.t >= 0 && r.t < count);
                    ++seen[(size_t)r.t];
                }
            for (int v : seen) REQUIRE(v == 1);
        }
    }
    std::printf("host planners: all checks passed\n");
    return 0;
}
