// Host-side entry points of the library exercised under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py with the
// sanitizers on the host pass only; nothing here touches a GPU).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ptycho.h"

static int failures = 0;
#define EXPECT(c)                                                               \
    do {                                                                        \
        if (!(c)) {                                                             \
            std::printf("FAILED %s line %d\n", #c, __LINE__);                  \
            ++failures;                                                         \
        }                                                                       \
    } while (0)

static std::vector<double> spiral(int j, double step) {
    std::vector<double> p(2 * (size_t)j);
    for (int i = 0; i < j; ++i) {
        const double r = step * std::sqrt((double)i), t = i * M_PI * (3.0 - std::sqrt(5.0));
        p[2 * i] = r * std::sin(t);
        p[2 * i + 1] = r * std::cos(t);
    }
    return p;
}

int main() {
    const int sizes[][6] = {  // n, K, J, ny, nx, step*10
        {16, 1, 37, 40, 56, 20}, {32, 2, 7, 64, 64, 30}, {64, 1, 100, 256, 256, 60},
        {128, 3, 21, 320, 288, 80}, {256, 3, 1000, 1024, 1024, 120}, {512, 4, 500, 2048, 2048, 240},
        {8, 2, 50, 48, 48, 10}, {1024, 2, 20, 1536, 1536, 400}};
    for (const auto &sz : sizes) {
        const int n = sz[0], k = sz[1], j = sz[2], ny = sz[3], nx = sz[4];
        std::vector<double> pos = spiral(j, sz[5] / 10.0);
        std::vector<int32_t> offs(2 * (size_t)j, -7);
        EXPECT(ptycho_offsets_from_positions(pos.data(), j, n, ny, nx, offs.data()) == PTYCHO_OK);
        for (int stack : {0, 1, 3, j / 2 + 1, j}) {
            for (uint32_t flags : {0u, (uint32_t)PTYCHO_FLAG_BACKGROUND, (uint32_t)PTYCHO_FLAG_POSITIONS}) {
                ptycho_desc_t d{n, k, j, ny, nx, stack, 0.01f, 0.01f, 1e-20f, flags};
                d.max_shift = 2.0f;
                size_t ws = 0, tb = 0;
                EXPECT(ptycho_workspace_bytes(&d, &ws) == PTYCHO_OK && ws > 0 && ws % 256 == 0);
                EXPECT(ptycho_plan_dry_run(&d, offs.data(), &tb) == PTYCHO_OK && tb > 0);
            }
        }
        // a window one pixel out of the object: an error, nothing written
        std::vector<double> bad = pos;
        bad[0] = ny / 2.0 - n / 2.0 + 0.5;
        std::vector<int32_t> o2(2 * (size_t)j, -7);
        EXPECT(ptycho_offsets_from_positions(bad.data(), j, n, ny, nx, o2.data()) == PTYCHO_E_BOUNDS);
        EXPECT(o2[0] == -7 && o2[2 * j - 1] == -7);
        EXPECT(std::strlen(ptycho_last_error()) > 0);
        std::vector<int32_t> o3 = offs;
        o3[2 * (j - 1)] = ny - n + 1;
        ptycho_desc_t d{n, k, j, ny, nx, 0, 0.01f, 0.01f, 1e-20f, 0};
        size_t tb = 0;
        EXPECT(ptycho_plan_dry_run(&d, o3.data(), &tb) == PTYCHO_E_BOUNDS);
    }
    // descriptor and argument errors
    ptycho_desc_t d{48, 1, 10, 128, 128, 0, 0.01f, 0.01f, 1e-20f, 0};
    size_t ws = 0;
    EXPECT(ptycho_workspace_bytes(&d, &ws) == PTYCHO_E_UNSUPPORTED);
    d.n = 64;
    d.flags = 8;
    EXPECT(ptycho_workspace_bytes(&d, &ws) == PTYCHO_E_INVALID);
    d.flags = PTYCHO_FLAG_POSITIONS;
    d.max_shift = -1.0f;
    EXPECT(ptycho_workspace_bytes(&d, &ws) == PTYCHO_E_INVALID);
    d.max_shift = 2.0f;
    EXPECT(ptycho_workspace_bytes(&d, &ws) == PTYCHO_OK);
    {
        // sub-pixel windows: corners and fractions, and a corner outside
        const double p2[4] = {0.25, -3.5, 100.0, 0.0};
        int32_t wo[4] = {-7, -7, -7, -7};
        double wf[4] = {-1, -1, -1, -1};
        EXPECT(ptycho_windows_from_positions(p2, 2, 64, 128, 128, wo, wf) == PTYCHO_E_BOUNDS);
        EXPECT(wo[0] == -7 && wf[0] == -1);
        const double p1[4] = {0.25, -3.5, 10.0, 0.0};
        EXPECT(ptycho_windows_from_positions(p1, 2, 64, 128, 128, wo, wf) == PTYCHO_OK);
        EXPECT(wo[0] == 32 && wo[1] == 28 && wf[0] == 0.25 && wf[1] == 0.5 && wo[2] == 42 && wf[2] == 0.0);
    }
    d.flags = PTYCHO_FLAG_NEAR_FIELD | PTYCHO_FLAG_BACKGROUND;
    size_t ws_nf = 0;
    EXPECT(ptycho_workspace_bytes(&d, &ws_nf) == PTYCHO_OK);
    d.flags = 0;
    EXPECT(ptycho_workspace_bytes(&d, &ws) == PTYCHO_OK);
    EXPECT(ws_nf >= ws + 2 * 64 * 8);
    EXPECT(ptycho_workspace_bytes(nullptr, &ws) == PTYCHO_E_INVALID);
    EXPECT(ptycho_plan_dry_run(&d, nullptr, &ws) == PTYCHO_E_INVALID);
    EXPECT(ptycho_plan_set_background(nullptr, nullptr) == PTYCHO_E_INVALID);
    EXPECT(ptycho_plan_set_near_field(nullptr, 0.1, 0.1) == PTYCHO_E_INVALID);
    EXPECT(ptycho_plan_timing(nullptr, 255) == PTYCHO_E_INVALID);
    std::printf("host checks: %d failures\n", failures);
    return failures == 0 ? 0 : 1;
}
