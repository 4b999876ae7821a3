// s3d_r1_f32.hip -- 3D radius-1 (7-point) streaming variants, FP32 storage.
#include "stream3d_impl.h"

namespace st {
namespace s3d {
static const Entry3 kTable[] = {
    S3D_BC(float, 1, 1, 4, 4, 4), S3D_BC(float, 1, 2, 4, 4, 4),
    S3D_BC(float, 1, 1, 4, 2, 8), S3D_BC(float, 1, 2, 4, 2, 8),
    S3D_BC(float, 1, 2, 4, 4, 8), S3D_BC(float, 1, 4, 4, 2, 8),
    S3D_BCL(float, 1, 3, 4, 4, 8, true), S3D_BCL(float, 1, 4, 4, 3, 8, true),
    S3D_BCY(float, 1, 2, 4, 4, 8, false), S3D_BCY(float, 1, 3, 4, 4, 8, true),
    S3D_BCY(float, 1, 3, 4, 5, 8, true), S3D_BCY(float, 1, 4, 4, 4, 8, true),
    S3D_FLUX(float, 1, 4, 4, 4, 8, true, true), S3D_FLUX(float, 1, 4, 4, 3, 8, true, false),
};
}  // namespace s3d

Table3 s3d_table_r1_f32() { return Table3{s3d::kTable, static_cast<int>(sizeof(s3d::kTable) / sizeof(s3d::kTable[0]))}; }

}  // namespace st
