// Stream-kernel variants, part 6 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart6[] = {
    SYNIM_VARIANT(256, 8, 3, 24, 6, 3),
    SYNIM_VARIANT_PACK(256, 4, 2, 8, 4, 3),
    SYNIM_VARIANT_PACK(256, 4, 3, 10, 4, 3),
    SYNIM_VARIANT_PACK(256, 4, 3, 10, 6, 3),
    SYNIM_VARIANT_PACK(256, 4, 3, 12, 4, 3),
};

const Variant* stream_variants_6(int* n) {
  *n = (int)(sizeof(kStreamPart6) / sizeof(kStreamPart6[0]));
  return kStreamPart6;
}

}  // namespace synim
