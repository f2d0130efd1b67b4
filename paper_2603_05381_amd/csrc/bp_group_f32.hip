// Group kernels of every size class with FP32 message storage.

#include "bp_group_impl.hpp"

namespace bpm {

int group_configs(int cls) { return configs_of(class_max_s(cls)).n; }

hipError_t launch_bp_group_f32(const DecodeShared &c, int cls, int cfg, hipStream_t stream) {
    return launch_group_ts<float>(c, cls, cfg, stream);
}

}  // namespace bpm
