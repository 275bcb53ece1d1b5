// Launch shapes recorded by the autotuner (paper_2604_08542_amd/tune.py) on MI355X; generated from
// tuned_tiles.json, do not edit.  Key: hidden size, BF16 operands, chunk tokens, chains, backward.
#pragma once
#include <stdint.h>

#include "../../include/ttt.h"

namespace ttt {
struct TunedShape {
  int32_t h, bf16;
  int64_t chunk_tokens, chains;
  int32_t bwd;
  ttt_tile_cfg_t cfg;
};
inline constexpr TunedShape kTuned[] = {
    {128, 1, 1374, 1, 0, {24, 0, 0, 0}},  // single_head_256x1374_bf16: 3.638 ms
    {128, 0, 1374, 1, 0, {0, 512, 1, 0}},  // single_head_4x1374: 0.122 ms
    {256, 1, 10992, 128, 0, {0, 0, 0, 0}},  // batch8_uneven_chunk8f_bf16: 7.400 ms
    {256, 1, 10992, 128, 1, {16, 0, 1, 0}},  // batch8_uneven_chunk8f_bf16: 43.296 ms
    {256, 1, 10992, 16, 0, {0, 256, 1, 0}},  // layer16_64f_chunk8f: 0.658 ms
    {256, 0, 10992, 16, 0, {16, 0, 1, 0}},  // layer16_64f_chunk8f: 2.867 ms
};
}  // namespace ttt
