// tune.hpp -- host-side declarations of the tuned-shape cache (tune.hip),
// shared by the batch and single-stack tuners.
#pragma once

#include <string>

#include "deskew.h"

namespace dsk {

// Tuned-shape cache (tune.hip): a JSON object in the file named by the
// DSK_TUNE_CACHE environment variable, one "key": {shape, "ms", "mode"}
// entry per line (mode: the batch execution mode, 0 for single stacks);
// without the variable nothing is read or written.  Keys begin with the
// device architecture (arch_name).
std::string arch_name();
bool tune_cache_lookup(const std::string &key, dsk_tune *t, double *ms, int *mode);
void tune_cache_store(const std::string &key, const dsk_tune &t, double ms, int mode);

}  // namespace dsk
