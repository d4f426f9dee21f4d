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
    {128, 128, 8},  // 0.811 ms
    {192, 192, 8},  // 1.106 ms
    {256, 256, 16},  // 1.324 ms
    {384, 384, 16},  // 1.972 ms
    {512, 512, 16},  // 2.847 ms
    {768, 768, 16},  // 5.142 ms
    {1024, 1024, 16},  // 8.831 ms
};
constexpr int kBatchTileTableSize = 7;

}  // namespace hyp
