/* Runs the CPU oracle (oracle/rcm_oracle.c, linked in) over the cases of a
 * binary file, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitizers.py), and prints one
 * line per case that the test compares with the ordinary build's results.
 *
 * Case file: repeated records of int32 values
 *   n nnz pp_variant reverse_mode full_check cm_mode rowptr[n+1] colidx[nnz]
 * (rowptr may be malformed: the oracle's validation is part of what runs).
 * Output line per case:
 *   status bw_before profile_before bw_after profile_after edges ncomp
 *   diameter nbfs nlevels perm[0..n-1] | iperm[0..n-1]
 * (only the status when it is not 0).
 *
 * usage: oracle_checks <case file> */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int64_t bandwidth_before;
    int64_t profile_before;
    int64_t bandwidth_after;
    int64_t profile_after;
    int64_t edges_traversed;
    int32_t num_components;
    int32_t pseudo_diameter;
    int32_t num_bfs;
    int32_t num_levels;
} orc_stats;

int orc_rcm_ex(int32_t n, const int32_t* rowptr, const int32_t* colidx, int pp_variant,
               int reverse_mode, int full_check, int cm_mode, int32_t* perm_out,
               int32_t* iperm_out, orc_stats* st, int32_t* comp_offset, int32_t* comp_root,
               int32_t* comp_nbfs, int32_t* comp_levels);

static int read_i32(FILE* f, int32_t* out, size_t count)
{
    return fread(out, sizeof(int32_t), count, f) == count;
}

int main(int argc, char** argv)
{
    if (argc < 2) {
        fprintf(stderr, "usage: %s <case file>\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) {
        perror(argv[1]);
        return 2;
    }
    int32_t head[6];
    int cases = 0;
    while (read_i32(f, head, 6)) {
        const int32_t n = head[0], nnz = head[1];
        if (n < 0 || nnz < 0) {
            fprintf(stderr, "case %d: bad sizes\n", cases);
            return 2;
        }
        /* exact-size buffers, so that any read past them is caught */
        int32_t* rowptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
        int32_t* colidx = (int32_t*)malloc(sizeof(int32_t) * (nnz > 0 ? (size_t)nnz : 1));
        int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? (size_t)n : 1));
        int32_t* iperm = (int32_t*)malloc(sizeof(int32_t) * (n > 0 ? (size_t)n : 1));
        if (!rowptr || !colidx || !perm || !iperm || !read_i32(f, rowptr, (size_t)n + 1) ||
            !read_i32(f, colidx, (size_t)nnz)) {
            fprintf(stderr, "case %d: truncated\n", cases);
            return 2;
        }
        orc_stats st;
        const int status = orc_rcm_ex(n, rowptr, colidx, head[2], head[3], head[4], head[5], perm,
                                      iperm, &st, NULL, NULL, NULL, NULL);
        printf("%d", status);
        if (status == 0) {
            printf(" %lld %lld %lld %lld %lld %d %d %d %d", (long long)st.bandwidth_before,
                   (long long)st.profile_before, (long long)st.bandwidth_after,
                   (long long)st.profile_after, (long long)st.edges_traversed,
                   st.num_components, st.pseudo_diameter, st.num_bfs, st.num_levels);
            for (int32_t k = 0; k < n; ++k) printf(" %d", perm[k]);
            printf(" |");
            for (int32_t k = 0; k < n; ++k) printf(" %d", iperm[k]);
        }
        printf("\n");
        free(rowptr);
        free(colidx);
        free(perm);
        free(iperm);
        ++cases;
    }
    fclose(f);
    fprintf(stderr, "%d cases\n", cases);
    return 0;
}
