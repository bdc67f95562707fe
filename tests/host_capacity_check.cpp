// Host-only driver of the library's capacity checks (csrc/capacity.hpp), built by
// tests/test_host_capacity.py with the host C++ compiler.  Prints one line per case.
#include <cstdio>

#include "../paper_2201_12663_amd/csrc/capacity.hpp"

int main() {
    struct Case { int m, zr_pad, p_cap; bool rf; int width, r, r_pad, want; };
    const Case cases[] = {
        {512, 512, 512, false, 0, 260, 384, 0},     // Gram-path fallback of the 512 x 1024 test
        {512, 512, 512, true, 64, 60, 128, 0},      // range finder within its width
        {512, 512, 512, true, 64, 65, 128, 4},      // rank beyond the sketch width
        {512, 512, 128, true, 192, 100, 128, 4},    // width beyond the test matrix
        {512, 512, 512, false, 0, 513, 640, 2},     // rank beyond m
        {1000, 1024, 512, false, 0, 1000, 1152, 3}, // padded rank beyond Z's columns
        {512, 512, 512, false, 0, 10, 100, 1},      // padding not a multiple of 128
        {2048, 2048, 2048, false, 0, 2048, 2048, 0},
    };
    int bad = 0;
    for (const Case& c : cases) {
        const int got = learned_mode_fits(c.m, c.zr_pad, c.p_cap, c.rf, c.width, c.r, c.r_pad);
        std::printf("m=%d r=%d r_pad=%d rf=%d width=%d -> %d (want %d)\n", c.m, c.r, c.r_pad, (int)c.rf, c.width, got,
                    c.want);
        bad += got != c.want;
    }
    return bad;
}
