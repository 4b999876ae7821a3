// s2d_bf16.hip -- 2D streaming-kernel variants with bf16s storage.
#include "stream2d_impl.h"

namespace st {
namespace s2d {
#define S2D_TB(CLS) S2D_BC(bf16s, 1, CLS, 1, 8), S2D_BC(bf16s, 1, CLS, 4, 8), S2D_BC(bf16s, 1, CLS, 8, 8)
static const Entry2 kTable[] = {S2D_TB(kStar), S2D_TB(kBox), S2D_FLUX(bf16s, 4, 8), S2D_FLUX(bf16s, 8, 8)};
}  // namespace s2d

Table2 s2d_table_bf16() { return Table2{s2d::kTable, static_cast<int>(sizeof(s2d::kTable) / sizeof(s2d::kTable[0]))}; }

}  // namespace st
