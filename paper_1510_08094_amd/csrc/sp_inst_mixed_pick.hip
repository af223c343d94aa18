#include "sp_inst_mixed.hpp"

sp::MixedSet sp::pick_mixed(int rs) {
    if (rs == kRadixFixed5000) return mixed_set_fixed();
    return rs <= 16 ? mixed_set_small() : mixed_set_large();
}
