// Cost-model and tile-cache files (persist.cpp).
#pragma once

#include <string>

#include "mlp.hpp"

namespace psc {

void mlp_file_write(const std::string &path, const MlpState &st);
MlpState mlp_file_read(const std::string &path);   // validated; throws PSC_ERR_IO
std::string tile_cache_key(int device);
void tile_cache_save(const std::string &path, const std::string &key);
int tile_cache_load(const std::string &path, const std::string &key);

}  // namespace psc
