// Stream-kernel variants, part 4 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart4[] = {
    SYNIM_VARIANT(512, 8, 2, 12, 3, 6),
    SYNIM_VARIANT(256, 8, 2, 12, 6, 3),
    SYNIM_VARIANT(1024, 8, 2, 14, 3, 3),
    SYNIM_VARIANT(512, 8, 2, 14, 3, 3),
    SYNIM_VARIANT(1024, 8, 2, 16, 3, 3),
};

const Variant* stream_variants_4(int* n) {
  *n = (int)(sizeof(kStreamPart4) / sizeof(kStreamPart4[0]));
  return kStreamPart4;
}

}  // namespace synim
