// s2d_f32.hip -- 2D streaming-kernel variants with float storage.
#include "stream2d_impl.h"

namespace st {
namespace s2d {
#define S2D_TB(CLS) S2D_BC(float, 1, CLS, 1, 4), S2D_BC(float, 1, CLS, 4, 4), S2D_BC(float, 1, CLS, 8, 4)
static const Entry2 kTable[] = {S2D_TB(kStar), S2D_TB(kBox), S2D_FLUX(float, 4, 4), S2D_FLUX(float, 8, 4)};
}  // namespace s2d

Table2 s2d_table_f32() { return Table2{s2d::kTable, static_cast<int>(sizeof(s2d::kTable) / sizeof(s2d::kTable[0]))}; }

}  // namespace st
