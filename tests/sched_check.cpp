// Host driver for the sanitizer test of the level schedule (schedule.h):
// reads patterns from a text file (per pattern: T nnzb, row_ptr, col_idx)
// and prints, per pattern, the status, then (status 0) the forward and
// backward level lists and offsets.  Built by tests/test_schedule_cpu.py
// with -fsanitize=address,undefined; test infrastructure only.
#include <cstdio>
#include <vector>

#include "schedule.h"

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int T, nnzb;
    while (std::fscanf(f, "%d %d", &T, &nnzb) == 2) {
        std::vector<int32_t> rp(T + 1 > 0 ? T + 1 : 1), ci(nnzb > 0 ? nnzb : 1);
        for (int i = 0; i <= T; ++i) if (std::fscanf(f, "%d", &rp[i]) != 1) return 2;
        for (int q = 0; q < nnzb; ++q) if (std::fscanf(f, "%d", &ci[q]) != 1) return 2;
        irk::Schedule sc;
        const int st = irk::analyze_pattern(T, nnzb, rp.data(), ci.data(), sc);
        std::printf("%d\n", st);
        if (st != 0) continue;
        for (const std::vector<int> *v : {&sc.lvl_fwd, &sc.off_fwd, &sc.lvl_bwd, &sc.off_bwd}) {
            for (int x : *v) std::printf("%d ", x);
            std::printf("\n");
        }
    }
    std::fclose(f);
    return 0;
}
