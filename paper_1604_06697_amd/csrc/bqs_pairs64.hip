// Kernel instantiations for key-value sorts with 64-bit payloads.
#include "bqs_kernels.hpp"

namespace bqs {

namespace {
template <int DT>
using Pairs = Launch<DT, uint64_t, 256, 16, 2048>;
}  // namespace

const Ops* ops_pairs64(int dtype) {
    switch (dtype) {
        case BQS_I32: return Pairs<BQS_I32>::ops();
        case BQS_U32: return Pairs<BQS_U32>::ops();
        case BQS_F32: return Pairs<BQS_F32>::ops();
        case BQS_I64: return Pairs<BQS_I64>::ops();
        case BQS_U64: return Pairs<BQS_U64>::ops();
        case BQS_F64: return Pairs<BQS_F64>::ops();
        default: return nullptr;
    }
}

}  // namespace bqs
