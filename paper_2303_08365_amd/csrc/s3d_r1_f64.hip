// s3d_r1_f64.hip -- 3D radius-1 (7-point) streaming variants, FP64 storage.
#include "stream3d_impl.h"

namespace st {
namespace s3d {
static const Entry3 kTable[] = {
    S3D_BC(double, 1, 1, 2, 4, 4), S3D_BC(double, 1, 2, 2, 4, 4),
    S3D_BC(double, 1, 1, 2, 2, 8), S3D_BC(double, 1, 2, 2, 2, 8),
    S3D_BC(double, 1, 2, 2, 4, 8), S3D_BC(double, 1, 4, 2, 2, 8),
    S3D_BCL(double, 1, 3, 2, 4, 8, true), S3D_BCL(double, 1, 4, 2, 3, 8, true),
    S3D_BCY(double, 1, 2, 2, 4, 8, false), S3D_BCY(double, 1, 3, 2, 4, 8, true),
    S3D_BCY(double, 1, 3, 2, 5, 8, true), S3D_BCY(double, 1, 4, 2, 4, 8, true),
    S3D_FLUX(double, 1, 4, 2, 4, 8, true, true),
};
}  // namespace s3d

Table3 s3d_table_r1_f64() { return Table3{s3d::kTable, static_cast<int>(sizeof(s3d::kTable) / sizeof(s3d::kTable[0]))}; }

}  // namespace st
