// Tile rows of the batched (streaming) Jacobi kernel per grid side: for
// batches of grids of nx x ny cells, the rows per wave R (8 or 16) that ran
// fastest on MI355X.  Written by paper_2109_09363_amd/autotune.py --batch
// (do not edit by hand); sides without an entry use R = 16.
#pragma once

namespace hyp {

struct BatchTileEntry {
  int nx, ny, R;
};

constexpr BatchTileEntry kBatchTileTable[] = {
    {128, 128, 8},  // 0.979 ms
    {192, 192, 16},  // 1.458 ms
    {256, 256, 16},  // 1.561 ms
    {384, 384, 16},  // 2.341 ms
    {512, 512, 16},  // 3.193 ms
};
constexpr int kBatchTileTableSize = 5;

}  // namespace hyp
