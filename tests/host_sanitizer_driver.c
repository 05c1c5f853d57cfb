/* Host-side paths of the library under AddressSanitizer and
 * UndefinedBehaviorSanitizer, with no GPU: argument checks that return
 * before any device work, the error-message buffer, the build id and the
 * tile cache's file parser fed valid, malformed and oversized files.
 * argv[1]: a directory for scratch files.  Exit status 0 on success; the
 * sanitizers abort the process on any report. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "spring_ising.h"

static int failures = 0;

#define EXPECT(cond)                                                \
  do {                                                              \
    if (!(cond)) {                                                  \
      fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond);   \
      ++failures;                                                   \
    }                                                               \
  } while (0)

static void write_file(const char *path, const char *text) {
  FILE *f = fopen(path, "w");
  if (!f) {
    fprintf(stderr, "cannot write %s\n", path);
    exit(2);
  }
  fputs(text, f);
  fclose(f);
}

int main(int argc, char **argv) {
  if (argc < 2) return 2;
  char path[4096], text[8192], head[256];
  const char *dir = argv[1];
  const char *id = spring_ising_build_id();
  EXPECT(id != NULL && strlen(id) > 0);

  /* parameters */
  si_params prm;
  EXPECT(spring_ising_default_params(NULL, 10) == SI_ERR_INVALID);
  EXPECT(spring_ising_default_params(&prm, 0) == SI_ERR_INVALID);
  EXPECT(strlen(spring_ising_last_error()) > 0);
  EXPECT(spring_ising_default_params(&prm, 10) == SI_OK);
  EXPECT(prm.total_steps == 10);

  /* entry points that reject their arguments before touching a device */
  EXPECT(spring_ising_init(NULL, 10, 4, NULL, NULL, NULL, &prm, NULL) == SI_ERR_INVALID);
  si_ctx *ctx = (si_ctx *)0;
  EXPECT(spring_ising_init(&ctx, 0, 4, NULL, NULL, NULL, &prm, NULL) == SI_ERR_INVALID);
  EXPECT(ctx == NULL);
  EXPECT(spring_ising_init_batch(&ctx, 0, NULL, 4, NULL, NULL, NULL, &prm, NULL) == SI_ERR_INVALID);
  EXPECT(spring_ising_destroy(NULL) == SI_OK);
  EXPECT(spring_ising_energy_noalloc(0, 4, NULL, NULL, NULL, NULL) == SI_ERR_INVALID);

  /* tile cache: a file of this build round-trips */
  snprintf(head, sizeof head, "# spring_ising tile cache 1\nbuild %s\n", id);
  EXPECT(spring_ising_tile_cache_clear() == SI_OK);
  snprintf(path, sizeof path, "%s/valid.txt", dir);
  snprintf(text, sizeof text,
           "%s0 0 11 0 1024 256 27 73.5\n1 5 19 12 64 256 2 905.25\n\n0 1 11 0 1024 256 32 17.1\n",
           head);
  write_file(path, text);
  int32_t n = -1;
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_OK && n == 3);
  snprintf(path, sizeof path, "%s/saved.txt", dir);
  EXPECT(spring_ising_tile_cache_save(path) == SI_OK);
  n = -1;
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_OK && n == 3);

  /* rejected files: nothing loaded, no memory error */
  const char *bad_bodies[] = {
      "0 0 11 0 1024 256 99 1\n",           /* no such FP32 tile */
      "1 0 19 12 64 256 3 1\n",             /* batch tiles are 1 and 2 */
      "0 0 11 0 1000 256 27 1\n",           /* R not a multiple of 64 */
      "0 0 11 0 1024 256 27\n",             /* missing field */
      "0 0 11 0 1024 256 27 1 extra\n",     /* trailing field */
      "-2147483648 0 0 0 0 0 0 0\n",        /* extreme integers */
      "99999999999999999999 0 0 0 64 1 1 1\n",
      "\x01\x02\x03\xff\xfe garbage\n",
  };
  for (size_t k = 0; k < sizeof bad_bodies / sizeof bad_bodies[0]; ++k) {
    snprintf(path, sizeof path, "%s/bad%zu.txt", dir, k);
    snprintf(text, sizeof text, "%s%s", head, bad_bodies[k]);
    write_file(path, text);
    n = -1;
    EXPECT(spring_ising_tile_cache_load(path, &n) == SI_ERR_INVALID && n == 0);
  }
  /* a line far longer than the parser's buffer */
  snprintf(path, sizeof path, "%s/long.txt", dir);
  {
    size_t off = (size_t)snprintf(text, sizeof text, "%s0 0 11 0 1024 256 27 ", head);
    while (off < sizeof text - 3) text[off++] = '7';
    text[off++] = '\n';
    text[off] = 0;
  }
  write_file(path, text);
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_ERR_INVALID);
  /* another build, another format, an empty file, a missing file */
  snprintf(path, sizeof path, "%s/other.txt", dir);
  write_file(path, "# spring_ising tile cache 1\nbuild 0000000000000000\n0 0 11 0 1024 256 27 1\n");
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_ERR_STATE);
  snprintf(path, sizeof path, "%s/magic.txt", dir);
  write_file(path, "# some other file\n");
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_ERR_INVALID);
  snprintf(path, sizeof path, "%s/empty.txt", dir);
  write_file(path, "");
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_ERR_INVALID);
  snprintf(path, sizeof path, "%s/absent.txt", dir);
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_ERR_INVALID);
  EXPECT(spring_ising_tile_cache_load(NULL, &n) == SI_ERR_INVALID);
  EXPECT(spring_ising_tile_cache_save(NULL) == SI_ERR_INVALID);
  snprintf(path, sizeof path, "%s/no_such_dir/x.txt", dir);
  EXPECT(spring_ising_tile_cache_save(path) == SI_ERR_INVALID);

  /* the cache still holds the three valid entries */
  snprintf(path, sizeof path, "%s/saved2.txt", dir);
  EXPECT(spring_ising_tile_cache_save(path) == SI_OK);
  n = -1;
  EXPECT(spring_ising_tile_cache_load(path, &n) == SI_OK && n == 3);
  EXPECT(spring_ising_tile_cache_clear() == SI_OK);

  if (failures) fprintf(stderr, "%d expectation(s) failed\n", failures);
  else printf("host sanitizer driver: all checks passed\n");
  return failures ? 1 : 0;
}
