/* Prints the C layout of the C-ABI descriptor structs; compiled by the host
 * test with gcc against include/kp.h and compared with the ctypes binding. */
#include <stddef.h>
#include <stdio.h>

#include "kp.h"

int main(void) {
  printf("kp_tensor %zu d %zu dtype %zu dims %zu data %zu\n", sizeof(kp_tensor),
         offsetof(kp_tensor, d), offsetof(kp_tensor, dtype), offsetof(kp_tensor, dims),
         offsetof(kp_tensor, data));
  printf("kp_matrix %zu rows %zu cols %zu rs %zu cs %zu dtype %zu data %zu\n", sizeof(kp_matrix),
         offsetof(kp_matrix, rows), offsetof(kp_matrix, cols), offsetof(kp_matrix, rs),
         offsetof(kp_matrix, cs), offsetof(kp_matrix, dtype), offsetof(kp_matrix, data));
  printf("enums %d %d %d %d %d %d %d %d %d %d %d\n", KP_OK, KP_ERR_NULL, KP_ERR_ORDER,
         KP_ERR_MODE, KP_ERR_SHAPE, KP_ERR_DTYPE, KP_ERR_ALIAS, KP_ERR_WORKSPACE, KP_ERR_HIP,
         KP_ERR_VALUE, KP_ERR_SCRATCH);
  printf("prec %d %d %d dtype %d %d maxorder %d\n", KP_PREC_NATIVE, KP_PREC_BF16X3,
         KP_PREC_BF16X6, KP_F64, KP_F32, KP_MAX_ORDER);
  printf("kp_tune_entry %zu form %zu Il %zu m %zu n %zu Ir %zu nb %zu fb %zu bk %zu occ %zu pf %zu\n",
         sizeof(kp_tune_entry), offsetof(kp_tune_entry, form), offsetof(kp_tune_entry, Il),
         offsetof(kp_tune_entry, m), offsetof(kp_tune_entry, n), offsetof(kp_tune_entry, Ir),
         offsetof(kp_tune_entry, nb), offsetof(kp_tune_entry, fb), offsetof(kp_tune_entry, bk),
         offsetof(kp_tune_entry, occ), offsetof(kp_tune_entry, pf));
  return 0;
}
