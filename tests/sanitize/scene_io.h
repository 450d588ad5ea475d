/* Raw scene arrays written by tests/test_sanitizers_cpu.py: DIR/meta.txt holds
 * "key value" lines (counts and scalars), DIR/<name>.bin each array. */
#ifndef SANITIZE_SCENE_IO_H
#define SANITIZE_SCENE_IO_H

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static long meta_get(const char *dir, const char *key) {
    char path[1024], k[128];
    long v;
    snprintf(path, sizeof path, "%s/meta.txt", dir);
    FILE *f = fopen(path, "r");
    if (!f) { fprintf(stderr, "no %s\n", path); exit(2); }
    while (fscanf(f, "%127s %ld", k, &v) == 2)
        if (strcmp(k, key) == 0) { fclose(f); return v; }
    fclose(f);
    fprintf(stderr, "no key %s in %s\n", key, path);
    exit(2);
}

/* the whole file, at least min_bytes long (exits otherwise); caller frees */
static void *read_bin(const char *dir, const char *name, long min_bytes) {
    char path[1024];
    snprintf(path, sizeof path, "%s/%s.bin", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) { fprintf(stderr, "no %s\n", path); exit(2); }
    fseek(f, 0, SEEK_END);
    long n = ftell(f);
    fseek(f, 0, SEEK_SET);
    if (n < min_bytes) { fprintf(stderr, "%s: %ld bytes, need %ld\n", path, n, min_bytes); exit(2); }
    void *p = malloc(n > 0 ? (size_t)n : 1);
    if (n > 0 && fread(p, 1, (size_t)n, f) != (size_t)n) { fprintf(stderr, "short read %s\n", path); exit(2); }
    fclose(f);
    return p;
}

#endif
