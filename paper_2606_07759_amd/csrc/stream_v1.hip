// Stream-kernel variants, part 1 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart1[] = {
    SYNIM_VARIANT(256, 4, 2, 8, 4, 3),
    SYNIM_VARIANT(256, 4, 2, 8, 4, 8),
    SYNIM_VARIANT(1024, 4, 3, 10, 3, 3),
    SYNIM_VARIANT(512, 4, 3, 10, 3, 6),
    SYNIM_VARIANT(512, 4, 3, 10, 2, 8),
};

const Variant* stream_variants_1(int* n) {
  *n = (int)(sizeof(kStreamPart1) / sizeof(kStreamPart1[0]));
  return kStreamPart1;
}

}  // namespace synim
