// s3d_r1_bf16.hip -- 3D radius-1 (7-point) streaming variants, bfloat16
// storage with FP32 compute.
#include "stream3d_impl.h"

namespace st {
namespace s3d {
static const Entry3 kTable[] = {
    S3D_BC(bf16s, 1, 1, 4, 4, 4), S3D_BC(bf16s, 1, 2, 4, 4, 4),
    S3D_BCY(bf16s, 1, 2, 4, 4, 8, false),
    S3D_FLUX(bf16s, 1, 2, 4, 4, 8, false, true),
};
}  // namespace s3d

Table3 s3d_table_r1_bf16() { return Table3{s3d::kTable, static_cast<int>(sizeof(s3d::kTable) / sizeof(s3d::kTable[0]))}; }

}  // namespace st
