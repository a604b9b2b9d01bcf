// Outcome counting of a step call (internal header): the fixed grid of the
// count kernel and the layout of its partial sums.
#pragma once

namespace adm1 {

// blocks of k_count_status (one per compute unit of the MI355X); block b
// stores its kFailSlots sums in row b of the context's partials, which the
// readout adds up
constexpr int kCountBlocks = 256;

}  // namespace adm1
