// Host-side check of the XCD slicing of a work-group order (no GPU needed): for the upper-triangle
// tile space of the pair-space polarization, every item of the order is dealt to exactly one
// work-group, and the 8 XCD slices hold working-item counts that differ by at most one.
// Prints one line per case: "ok <cases fields>" or "FAIL ...".
#include "../../paper_1602_02313_amd/csrc/k_mfma.hip"

#include <cstdio>

namespace msgw {
namespace {
int check(int NI, int WI, int SR, int SC, int nq, int ntc) {
    const int R = ceil_div(NI, 4 * WI), C = ceil_div(NI, 16) * ntc;
    const Order od = make_order_st(R, C, nq, SR, SC * ntc);
    auto rows = [&](int, int r, int& lo, int& hi) {
        const int I0 = r * 4 * WI;
        lo = I0 / 16 * ntc;
        hi = I0 < NI ? ceil_div(NI, 16) * ntc : lo;
    };
    int bad = -1;
    try {
        launch_order(od, 128 * WI, [&](dim3 g, const Order& o) {
            std::vector<int> seen(o.n, 0);
            int cnt[8] = {0};
            for (unsigned b = 0; b < g.x; ++b) {
                const int x = b & 7;
                const int w = o.xs[x] + int(b >> 3);
                if (w >= o.xs[x + 1]) continue;
                ++seen[w];
                int qrel, r, c;
                order_item(o, w + o.off, qrel, r, c);
                if (r >= o.R || c >= o.C) continue;
                const int I0 = r * 4 * WI, J0 = (c / ntc) * 16;
                if (I0 < NI && J0 < NI && J0 + 16 > I0) ++cnt[x];
            }
            int once = 0, lo = 1 << 30, hi = 0, tot = 0;
            for (int v : seen) once += v == 1;
            for (int x = 0; x < 8; ++x) {
                lo = std::min(lo, cnt[x]);
                hi = std::max(hi, cnt[x]);
                tot += cnt[x];
            }
            const int64_t counted = order_count(o, o.off, int64_t(o.off) + o.n, rows);
            bad = (once != o.n || hi - lo > 1 || tot != counted) ? 1 : 0;
            std::printf("%s NI=%d WI=%d st=%dx%d nq=%d ntc=%d items=%d covered=%d working=%d per-XCD=%d..%d\n",
                        bad ? "FAIL" : "ok", NI, WI, SR, SC, nq, ntc, o.n, once, tot, lo, hi);
        }, rows);
    } catch (const std::exception&) {
        // launch_order checks the (absent) device after the launch callback; the callback has run
    }
    return bad;
}
}  // namespace
}  // namespace msgw

int main() {
    int fails = 0;
    const int cases[][6] = {{400, 4, 4, 8, 4, 1}, {400, 4, 4, 8, 16, 1}, {400, 2, 4, 16, 4, 1}, {333, 4, 4, 8, 3, 2},
                            {57, 4, 4, 8, 5, 1},  {16, 4, 4, 8, 1, 3},   {900, 4, 4, 8, 1, 2},  {1000, 2, 4, 16, 7, 1}};
    for (const auto& c : cases) fails += msgw::check(c[0], c[1], c[2], c[3], c[4], c[5]) != 0;
    return fails;
}
