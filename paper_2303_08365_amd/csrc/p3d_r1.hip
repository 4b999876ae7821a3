// p3d_r1.hip -- 3D radius-1 (7-point) partial-sum pipeline variants
// (pipe3d_impl.h): up to four fused steps, whole-vector rows; input planes
// one ahead in registers or two ahead through the LDS queue.
#include "pipe3d_impl.h"

namespace st {
namespace p3d {
static const Entry3 kTable[] = {
    P3D_BC(double, 4, 2, 4, 8, 2, 1),
    P3D_BC(double, 4, 2, 4, 8, 1, 1),
    P3D_BC(double, 4, 2, 3, 8, 2, 1),
    P3D_BC(double, 3, 2, 4, 8, 2, 1),
    P3D_BC(float, 4, 2, 8, 8, 2, 1),
    P3D_BC(float, 4, 4, 4, 8, 2, 1),
    P3D_BC(float, 4, 4, 4, 8, 1, 1),
    P3D_BC(float, 4, 4, 3, 8, 2, 1),
    P3D_BC(float, 3, 4, 4, 8, 2, 1),
    P3D_BC(bf16s, 4, 4, 4, 8, 2, 1),
    P3D_BC(bf16s, 3, 4, 4, 8, 2, 1),
    P3D_BC(bf16s, 3, 4, 6, 8, 2, 1),
    P3D_LQ(double, 4, 2, 8),
    P3D_LQ(float, 4, 4, 8),
    P3D_FLUX(double, 4, 2, 4, 8, 2, 1),
    P3D_FLUX(float, 4, 4, 4, 8, 2, 1),
    P3D_FLUX(bf16s, 3, 4, 4, 8, 2, 1),
    P3D_LQ_FLUX(double, 4, 2, 8),
    P3D_LQ_FLUX(float, 4, 4, 8),
};
}  // namespace p3d

Table3 p3d_table_r1() { return Table3{p3d::kTable, static_cast<int>(sizeof(p3d::kTable) / sizeof(p3d::kTable[0]))}; }

}  // namespace st
