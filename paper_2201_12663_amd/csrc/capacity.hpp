// Host-side capacity checks (no HIP types: also compiled by the host-only tests).
#pragma once

// Buffers of one mode of the learned path's reduction: Z^(l) holds zr_pad columns
// (zr_pad = min(n, R) rounded up to 128), the range finder's selection matrix
// p_cap x zr_pad.  A rank r (padded to r_pad, a multiple of 128) fits when
// r <= m, r_pad <= zr_pad, and on a range-finder mode of width p, 1 <= p <= p_cap
// and r <= p.  Returns 0 when it fits, else the number of the failed condition.
inline int learned_mode_fits(int m, int zr_pad, int p_cap, bool range_finder, int width, int r, int r_pad) {
    if (r < 0 || r_pad < r || r_pad % 128 != 0) return 1;
    if (r > m) return 2;
    if (r_pad > zr_pad) return 3;
    if (range_finder && (width < 1 || width > p_cap || r > width)) return 4;
    return 0;
}
