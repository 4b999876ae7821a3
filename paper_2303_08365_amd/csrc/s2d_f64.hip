// s2d_f64.hip -- 2D streaming-kernel variants with double storage.
#include "stream2d_impl.h"

namespace st {
namespace s2d {
#define S2D_TB(CLS) S2D_BC(double, 1, CLS, 1, 2), S2D_BC(double, 1, CLS, 4, 2), S2D_BC(double, 1, CLS, 8, 2)
static const Entry2 kTable[] = {S2D_TB(kStar), S2D_TB(kBox), S2D_FLUX(double, 4, 2), S2D_FLUX(double, 8, 2)};
}  // namespace s2d

Table2 s2d_table_f64() { return Table2{s2d::kTable, static_cast<int>(sizeof(s2d::kTable) / sizeof(s2d::kTable[0]))}; }

}  // namespace st
