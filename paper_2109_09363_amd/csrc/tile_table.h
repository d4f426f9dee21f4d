// Tuned tile heights of the persistent Jacobi kernel: for a grid of
// nx x ny cells and halo H, the rows per wave R that ran fastest on MI355X.
// Written by paper_2109_09363_amd/autotune.py (do not edit by hand); a grid
// without an entry uses the smallest R whose tiles fit one work-group per CU.
#pragma once

namespace hyp {

struct TileEntry {
  int nx, ny, H, R;
};

constexpr TileEntry kTileTable[] = {
    {128, 128, 9, 8},  // 0.373 ms
    {192, 192, 9, 8},  // 0.376 ms
    {256, 256, 9, 8},  // 0.383 ms
    {384, 384, 9, 8},  // 0.395 ms
    {512, 512, 9, 12},  // 0.459 ms
    {768, 768, 9, 24},  // 0.647 ms
    {1024, 1024, 9, 32},  // 0.811 ms
};
constexpr int kTileTableSize = 7;

}  // namespace hyp
