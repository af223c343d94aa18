#include "sp_inst_mixed.hpp"

sp::MixedSet sp::mixed_set_fixed() { return mixed_set<kRadixFixed5000>(); }
