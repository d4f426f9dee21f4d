// Tile rows of the batched (streaming) Jacobi kernel per grid side: for
// batches of grids of nx x ny cells, the rows per wave R (8 or 16) that ran
// fastest on MI355X.  Written by paper_2109_09363_amd/autotune.py --batch
// (do not edit by hand); sides without an entry use R = 16.
#pragma once

namespace hyp {

struct BatchTileEntry {
  int nx, ny, R;
};

// (no measured entries yet)
constexpr BatchTileEntry kBatchTileTable[] = {{0, 0, 16}};
constexpr int kBatchTileTableSize = 0;

}  // namespace hyp
