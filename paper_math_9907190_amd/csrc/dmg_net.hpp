// Host-side helpers of the learned coarse correction shared by the trainer
// and the plans that run the network inside their coarse kernels.
#pragma once
#include "dmg_net_dev.hpp"

namespace dmg {

// logical weights of the network in `dim` dimensions (0 for another dim)
int net_weight_count(int dim);
// fp32 weights [layer][tap][ci][co] -> packed bf16 forward / input-gradient forms of
// NetGeo<dim>::PACK entries each, padding zeroed (either may be null)
void net_pack_host(int dim, const float* w, bf16_t* wf, bf16_t* wb);

}  // namespace dmg
