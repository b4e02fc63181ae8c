// Library calls the request loop uses beyond the public boundary.
#pragma once

#include "hwpm.h"

namespace hwpm {

// The first half of hwpm_match_batch alone: every block's perfect matching
// (greedy proposals, then augmenting paths) into its perm_out, item status
// HWPM_OK, or HWPM_ESINGULAR with perm_out untouched; no rounds.  The
// workspace is hwpm_batch_workspace_bytes of the batch.  The request loop
// improves these matchings later, in round batches shared with the requests
// already in flight.
int match_batch_initial(hwpm_handle h, int32_t count, const hwpm_csc* mats, int32_t* const* perm_out,
                        const hwpm_options* opt, hwpm_item_stats* items, void* workspace,
                        size_t workspace_bytes);

}  // namespace hwpm
