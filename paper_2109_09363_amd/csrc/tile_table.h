// Tuned tiles of the persistent Jacobi kernel: for a grid of nx x ny cells,
// the halo H (H - 1 sweeps between exchanges) and rows per wave R that ran
// fastest on MI355X.  Written by paper_2109_09363_amd/autotune.py (do not
// edit by hand); a grid without an entry uses H = 9 and the smallest R
// whose tiles fit one work-group per CU.
#pragma once

namespace hyp {

struct TileEntry {
  int nx, ny, H, R;
};

constexpr TileEntry kTileTable[] = {
    {128, 128, 17, 12},  // 1.014 ms
    {192, 192, 17, 12},  // 1.015 ms
    {256, 256, 17, 12},  // 1.030 ms
    {384, 384, 17, 16},  // 1.163 ms
    {512, 512, 9, 8},  // 1.245 ms
    {768, 768, 13, 24},  // 2.024 ms
    {1024, 1024, 9, 32},  // 2.772 ms
};
constexpr int kTileTableSize = 7;

}  // namespace hyp
