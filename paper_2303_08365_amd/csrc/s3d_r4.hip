// s3d_r4.hip -- 3D radius-4 (25-point) streaming variants, one fused step.
#include "stream3d_impl.h"

namespace st {
namespace s3d {
static const Entry3 kTable[] = {
    S3D_BC(float, 4, 1, 4, 2, 8), S3D_BC(float, 4, 1, 4, 1, 16),
    S3D_BC(double, 4, 1, 4, 1, 8), S3D_BC(bf16s, 4, 1, 4, 2, 8),
    S3D_BCY(float, 4, 1, 4, 2, 8, false), S3D_BCY(float, 4, 1, 4, 1, 16, false),
    S3D_BCY(double, 4, 1, 4, 1, 8, false), S3D_BCY(bf16s, 4, 1, 4, 2, 8, false),
};
}  // namespace s3d

Table3 s3d_table_r4() { return Table3{s3d::kTable, static_cast<int>(sizeof(s3d::kTable) / sizeof(s3d::kTable[0]))}; }

}  // namespace st
