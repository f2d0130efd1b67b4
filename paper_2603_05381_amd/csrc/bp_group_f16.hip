// Group kernels of every size class with FP16 message storage.

#include "bp_group_impl.hpp"

namespace bpm {

hipError_t launch_bp_group_f16(const DecodeShared &c, int cls, int cfg, hipStream_t stream) {
    return launch_group_ts<_Float16>(c, cls, cfg, stream);
}

}  // namespace bpm
