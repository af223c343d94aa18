// Kernel builds of the single-problem mixed-precision passes, one radix set
// per translation unit (sp_inst_mixed_*.hip; see sp_tables.hpp).
#pragma once
#include "sp_tables.hpp"

namespace sp {
template <int RMAX>
MixedSet mixed_set() {
    MixedSet k{{nullptr, &k_theta_mixed_real<kEPT, RMAX, kSmaxR, kSmaxR, false, false>},
               {nullptr, &k_theta_mixed_real<kEPT, RMAX, kSmaxR, kSmaxR, true, false>},
               {nullptr, &k_theta_mixed_real<kEPT, RMAX, kSmaxR, kSmaxR, false, true>},
               {nullptr, &k_theta_mixed_real<kEPT, RMAX, kSmaxR, kSmaxR, true, true>},
               {nullptr, &k_theta_mixed_real<kEPT, RMAX, kSmaxR, kSmaxR, true, false, true>},
               {nullptr, &k_theta_mixed_real<kEPT, RMAX, kSmaxR, kSmaxR, true, true, true>},
               &k_lambda_mix<kEPT, RMAX>, &k_lambda_update<kEPT, RMAX>};
    if constexpr (RMAX != kRadixFixed5000) {
        k.theta_first[0] = &k_theta_mixed<kEPT, RMAX, kSmaxF, kSmaxD, false, false>;
        k.theta_resid[0] = &k_theta_mixed<kEPT, RMAX, kSmaxF, kSmaxD, true, false>;
        k.theta_first_t[0] = &k_theta_mixed<kEPT, RMAX, kSmaxF, kSmaxD, false, true>;
        k.theta_resid_t[0] = &k_theta_mixed<kEPT, RMAX, kSmaxF, kSmaxD, true, true>;
        k.theta_resid_norm[0] = &k_theta_mixed<kEPT, RMAX, kSmaxF, kSmaxD, true, false, true>;
        k.theta_resid_t_norm[0] = &k_theta_mixed<kEPT, RMAX, kSmaxF, kSmaxD, true, true, true>;
    }
    return k;
}
MixedSet mixed_set_small();   // radices up to 16
MixedSet mixed_set_large();   // radices up to 31
MixedSet mixed_set_fixed();   // the fixed length-5000 transform
}  // namespace sp
