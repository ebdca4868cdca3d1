// Stream-kernel variants, part 0 of the table (see stream.hpp).
#include "stream.hpp"

namespace synim {

const Variant kStreamPart0[] = {
    SYNIM_VARIANT(1024, 4, 2, 8, 3, 3),
    SYNIM_VARIANT(512, 4, 2, 8, 3, 6),
    SYNIM_VARIANT(512, 4, 2, 8, 3, 3),
    SYNIM_VARIANT(512, 4, 3, 10, 3, 3),
    SYNIM_VARIANT(512, 4, 3, 12, 3, 3),
};

const Variant* stream_variants_0(int* n) {
  *n = (int)(sizeof(kStreamPart0) / sizeof(kStreamPart0[0]));
  return kStreamPart0;
}

}  // namespace synim
