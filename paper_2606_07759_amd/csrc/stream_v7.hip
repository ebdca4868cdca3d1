// Stream-kernel variants, part 7 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart7[] = {
    SYNIM_VARIANT_PACK(256, 8, 2, 12, 6, 3),
    SYNIM_VARIANT_PACK(256, 8, 2, 14, 6, 3),
    SYNIM_VARIANT_PACK(256, 8, 2, 16, 6, 3),
    SYNIM_VARIANT_PACK(256, 8, 3, 20, 6, 3),
    SYNIM_VARIANT_PACK(256, 8, 3, 24, 6, 3),
};

const Variant* stream_variants_7(int* n) {
  *n = (int)(sizeof(kStreamPart7) / sizeof(kStreamPart7[0]));
  return kStreamPart7;
}

}  // namespace synim
