/* Prints the size and field offsets of the public structs (C compiler view). */
#include <stddef.h>
#include <stdio.h>

#include "degrid.h"

int main(void) {
    printf("{\"dg_desc\": [%zu, %zu, %zu, %zu, %zu, %zu], ", sizeof(dg_desc), offsetof(dg_desc, os_uv),
           offsetof(dg_desc, grid_dtype), offsetof(dg_desc, n_b), offsetof(dg_desc, flags),
           offsetof(dg_desc, support_w));
    printf("\"dg_plan_info\": [%zu, %zu, %zu, %zu, %zu, %zu, %zu]}\n", sizeof(dg_plan_info),
           offsetof(dg_plan_info, n_tiles), offsetof(dg_plan_info, n_b), offsetof(dg_plan_info, n_queues),
           offsetof(dg_plan_info, device), offsetof(dg_plan_info, sorted), offsetof(dg_plan_info, n_kernels));
    return 0;
}
