#include "sp_inst_mixed.hpp"

sp::MixedSet sp::mixed_set_small() { return mixed_set<16>(); }
