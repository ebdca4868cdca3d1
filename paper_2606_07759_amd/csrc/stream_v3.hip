// Stream-kernel variants, part 3 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart3[] = {
    SYNIM_VARIANT(256, 4, 3, 10, 3, 3),
    SYNIM_VARIANT(256, 4, 3, 10, 6, 3),
    SYNIM_VARIANT(1024, 4, 3, 12, 3, 3),
    SYNIM_VARIANT(512, 4, 3, 12, 3, 6),
    SYNIM_VARIANT(256, 4, 3, 12, 4, 3),
};

const Variant* stream_variants_3(int* n) {
  *n = (int)(sizeof(kStreamPart3) / sizeof(kStreamPart3[0]));
  return kStreamPart3;
}

}  // namespace synim
