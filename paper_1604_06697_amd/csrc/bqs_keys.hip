// Kernel instantiations for key-only sorts.
#include "bqs_kernels.hpp"

namespace bqs {

namespace {
template <int DT, int EPT>
using Keys4 = Launch<DT, NoVal, 256, EPT, 16384>;  // 4-byte keys: small segments up to 16384 keys
template <int DT>
using Keys8 = Launch<DT, NoVal, 256, 16, 4096>;   // 8-byte keys: 32 KB small-sort LDS

template <int DT>
const Ops* four_byte(int ept) {
    switch (ept) {
        case 8: return Keys4<DT, 8>::ops();
        case 16: return Keys4<DT, 16>::ops();
        default: return Keys4<DT, 32>::ops();
    }
}
}  // namespace

const Ops* ops_keys(int dtype, int ept) {
    switch (dtype) {
        case BQS_I32: return four_byte<BQS_I32>(ept);
        case BQS_U32: return Keys4<BQS_U32, 32>::ops();
        case BQS_F32: return Keys4<BQS_F32, 32>::ops();
        case BQS_I64: return Keys8<BQS_I64>::ops();
        case BQS_U64: return Keys8<BQS_U64>::ops();
        case BQS_F64: return Keys8<BQS_F64>::ops();
        default: return nullptr;
    }
}

}  // namespace bqs
