// Reduced-precision rank-K kernels (FP32 and BF16x3).  Not yet available:
// the tile tables are empty, so the API reports CHI0_EUNSUPPORTED.
#include "common.h"
#include "herk_common.h"

namespace chi0 {
int herk_fp32_tile_count() { return 0; }
TileConfig herk_fp32_tile(int) { return TileConfig{0, 0, 0, 0}; }
hipError_t herk_fp32_launch(int, const HerkArgs&, int, hipStream_t) { return hipErrorInvalidValue; }
int herk_fp32_max_wg_per_cu(int) { return 1; }
int herk_bf16x3_tile_count() { return 0; }
TileConfig herk_bf16x3_tile(int) { return TileConfig{0, 0, 0, 0}; }
hipError_t herk_bf16x3_launch(int, const HerkArgs&, int, hipStream_t) { return hipErrorInvalidValue; }
int herk_bf16x3_max_wg_per_cu(int) { return 1; }
}  // namespace chi0
