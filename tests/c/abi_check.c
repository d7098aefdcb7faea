/* Compiled as C11 against include/tw.h and linked with libtw.so by
 * tests/test_c_abi.py: the header is plain C, the layouts the ctypes binding
 * assumes are the compiler's, and the host-only entry points run from C. */
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>

#include "tw.h"

int main(void)
{
    printf("sizeof_options %zu\n", sizeof(tw_options));
    printf("off_reductions %zu\n", offsetof(tw_options, reductions));
    printf("off_mmw_prune %zu\n", offsetof(tw_options, mmw_prune));
    printf("off_batch_schedule %zu\n", offsetof(tw_options, batch_schedule));
    printf("off_batch_chunk %zu\n", offsetof(tw_options, batch_chunk));
    printf("off_workspace %zu\n", offsetof(tw_options, workspace));
    printf("off_workspace_bytes %zu\n", offsetof(tw_options, workspace_bytes));
    printf("off_fault_inject_level %zu\n", offsetof(tw_options, fault_inject_level));
    printf("off_capture %zu\n", offsetof(tw_options, capture));
    printf("sizeof_batch_level %zu\n", sizeof(tw_batch_level));
    printf("sizeof_stats %zu\n", sizeof(tw_stats));
    printf("sizeof_graph_stats %zu\n", sizeof(tw_graph_stats));
    printf("sizeof_graph %zu\n", sizeof(tw_graph));
    printf("sizeof_level_record %zu\n", sizeof(tw_level_record));

    /* a 5-cycle: treewidth 2 */
    uint64_t rows[5];
    for (int i = 0; i < 5; ++i)
        rows[i] = (1ull << ((i + 1) % 5)) | (1ull << ((i + 4) % 5));
    tw_graph g = {5, rows};
    int32_t lb = -1, width = -1;
    if (tw_mmw(&g, &lb) != TW_OK)
        return 1;
    int32_t order[5] = {0, 1, 2, 3, 4};
    if (tw_order_width(&g, order, &width) != TW_OK)
        return 2;
    uint64_t bags[5];
    int32_t parent[5], dwidth = -1;
    if (tw_tree_decomposition(&g, order, bags, parent, &dwidth) != TW_OK)
        return 3;
    uint64_t clique = 0;
    if (tw_reductions(&g, &clique, NULL) != TW_OK)
        return 4;
    printf("mmw %d width %d decomposition_width %d clique_bits %d\n", lb, width, dwidth,
           __builtin_popcountll(clique));
    printf("status_str %s\n", tw_status_str(TW_EINVAL));
    return 0;
}
