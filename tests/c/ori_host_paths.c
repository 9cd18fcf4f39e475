/* Host-only paths of the C ABI (no device needed): version and defaults,
 * workspace sizes, the argument checks of ori_create and the out-of-memory
 * refusal before any device call, error texts.  Built with the runtime's
 * host code under AddressSanitizer and UBSan (see build.py); exit status 0
 * and a line "OK 0" on success. */
#include <stdio.h>
#include <string.h>
#include "ori.h"
int main(void) {
  int bad = 0;
  printf("%s\n", ori_version());
  ori_solve_opts o;
  ori_default_opts(&o);
  for (int n = 1; n <= 512; n *= 2) {
    ori_grid gg = {n, 1.0, {0, 0, 0}, 0.5};
    int64_t b = 0;
    if (ori_workspace_bytes(&gg, 1, 3, &b) != ORI_OK || b <= 0) bad++;
  }
  ori_grid g = {513, 1.0, {0, 0, 0}, 0.5};  /* beyond the largest planned length */
  ori_ctx c = NULL;
  if (ori_create(&g, 1, 3, 0, NULL, &c) == ORI_OK) bad++;
  if (strlen(ori_last_error(NULL)) == 0) bad++;
  g.n = 0;
  if (ori_create(&g, 1, 3, 0, NULL, &c) == ORI_OK) bad++;
  g.n = 8; g.side = -1.0;
  if (ori_create(&g, 1, 3, 0, NULL, &c) == ORI_OK) bad++;
  if (ori_create(NULL, 1, 3, 0, NULL, &c) == ORI_OK) bad++;
  g.side = 1.0;
  if (ori_create(&g, 0, 3, 0, NULL, &c) == ORI_OK) bad++;
  ori_status st = ori_create(&g, 1, 3, 1024, NULL, &c);  /* memory limit below the workspace */
  if (st != ORI_ERR_OUT_OF_MEMORY) bad++;
  ori_destroy(NULL);
  printf("%s %d\n", bad ? "FAIL" : "OK", bad);
  return bad != 0;
}
