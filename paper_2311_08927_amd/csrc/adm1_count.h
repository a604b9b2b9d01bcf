// Outcome counting of a step call (internal header): the fixed grid of the
// count kernel and the layout of its partial sums.
#pragma once

namespace adm1 {

// blocks of k_count_status; block b stores its kFailSlots sums in row b of
// the context's partials, which the readout adds up
constexpr int kCountBlocks = 64;

}  // namespace adm1
