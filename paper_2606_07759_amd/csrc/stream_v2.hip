// Stream-kernel variants, part 2 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart2[] = {
    SYNIM_VARIANT(256, 4, 3, 10, 4, 3),
    SYNIM_VARIANT(256, 4, 3, 10, 4, 8),
    SYNIM_VARIANT(256, 4, 3, 10, 3, 4),
    SYNIM_VARIANT(256, 4, 3, 10, 4, 4),
    SYNIM_VARIANT(256, 4, 3, 10, 3, 5),
};

const Variant* stream_variants_2(int* n) {
  *n = (int)(sizeof(kStreamPart2) / sizeof(kStreamPart2[0]));
  return kStreamPart2;
}

}  // namespace synim
