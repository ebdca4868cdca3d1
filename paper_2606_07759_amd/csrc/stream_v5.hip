// Stream-kernel variants, part 5 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart5[] = {
    SYNIM_VARIANT(512, 8, 2, 14, 3, 6),
    SYNIM_VARIANT(256, 8, 2, 14, 6, 3),
    SYNIM_VARIANT(512, 8, 2, 16, 3, 6),
    SYNIM_VARIANT(256, 8, 2, 16, 6, 3),
    SYNIM_VARIANT(256, 8, 3, 20, 6, 3),
};

const Variant* stream_variants_5(int* n) {
  *n = (int)(sizeof(kStreamPart5) / sizeof(kStreamPart5[0]));
  return kStreamPart5;
}

}  // namespace synim
