#include "sp_inst_mixed.hpp"

sp::MixedSet sp::mixed_set_large() { return mixed_set<32>(); }
