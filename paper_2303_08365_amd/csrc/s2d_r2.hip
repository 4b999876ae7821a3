// s2d_r2.hip -- 2D radius-2 stars (9 points) and boxes (25 points), FP64,
// FP32 and bfloat16 storage; one step or up to four fused steps.
#include "stream2d_impl.h"

namespace st {
namespace s2d {
#define S2D_R2(TS, VX) \
    S2D_BC(TS, 2, kStar, 1, VX), S2D_BC(TS, 2, kStar, 4, VX), S2D_BC(TS, 2, kBox, 1, VX), S2D_BC(TS, 2, kBox, 4, VX)
static const Entry2 kTable[] = {S2D_R2(double, 2), S2D_R2(float, 4), S2D_R2(bf16s, 8)};
}  // namespace s2d

Table2 s2d_table_r2() { return Table2{s2d::kTable, static_cast<int>(sizeof(s2d::kTable) / sizeof(s2d::kTable[0]))}; }

}  // namespace st
