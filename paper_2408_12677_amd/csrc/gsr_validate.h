// Argument validation of the C ABI, in plain C++17 with no HIP dependency: every public
// entry point checks its host-side arguments with these before any device work, and the
// host test-suite builds this file (with the keyframe schedule, the other host-only unit)
// under the address and undefined-behaviour sanitizers.  Each check returns GSR_OK or an
// error status with a message in `err`.
#ifndef GSR_VALIDATE_H
#define GSR_VALIDATE_H

#include <string>

#include "gsr.h"

namespace gsr {
namespace check {

gsr_status settings(const gsr_settings* s, std::string& err);
gsr_status gaussians(const gsr_gaussians* g, int views, std::string& err);
gsr_status camera(const gsr_camera& c, int view, std::string& err);
// cams[V] and outs[V]: the sizes, rules and every view's camera and colour output.
gsr_status forward_args(const gsr_gaussians* g, const gsr_camera* cams, int32_t V, const gsr_settings* s,
                        const gsr_view_out* outs, std::string& err);
// The optimiser's moments, state word and rates.
gsr_status adam(const gsr_adam* o, std::string& err);
gsr_status seed_settings(const gsr_seed_settings* s, int64_t capacity, const gsr_seed_out* out, std::string& err);
// TSDF map settings and capacity; *slots receives the hash-table size (a power of two
// >= 2 max_blocks, at least 1024).
gsr_status tsdf_settings(const gsr_tsdf_settings* s, int64_t max_blocks, int64_t* slots, std::string& err);

}  // namespace check
}  // namespace gsr

#endif  // GSR_VALIDATE_H
