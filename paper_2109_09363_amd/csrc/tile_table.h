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
    {128, 128, 13, 12},  // 0.822 ms
    {192, 192, 13, 12},  // 0.828 ms
    {256, 256, 13, 12},  // 0.850 ms
    {384, 384, 13, 12},  // 0.912 ms
    {512, 512, 17, 16},  // 0.983 ms
    {768, 768, 13, 24},  // 1.919 ms
    {1024, 1024, 9, 32},  // 2.622 ms
};
constexpr int kTileTableSize = 7;

}  // namespace hyp
