// corr_tune.h -- launch-shape cache shared by corr_create and corr_autotune.
#ifndef CORR_TUNE_H
#define CORR_TUNE_H

#include <string>

#include "../../include/corr.h"

namespace corr {

std::string tune_cache_path(const char *explicit_path);
std::string tune_key(const corr_group_desc *g, int n, uint32_t flags, int device);
bool tune_cache_lookup(const std::string &path, const std::string &key, corr_tuning *out);

} // namespace corr

#endif
