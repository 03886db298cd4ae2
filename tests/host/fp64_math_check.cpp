// Host build of the cell models' FP64 exponential and logarithm: reads
// binary doubles from the file named by argv[2], writes exp64 (argv[1] =
// "exp") or log64 ("log") of each to the file named by argv[3].
#include "cellmodels.hpp"
#include <cstdio>
#include <cstring>
#include <vector>

int main(int argc, char **argv) {
    if (argc != 4) return 2;
    const bool is_exp = std::strcmp(argv[1], "exp") == 0;
    if (!is_exp && std::strcmp(argv[1], "log") != 0) return 2;
    FILE *f = std::fopen(argv[2], "rb");
    if (!f) return 3;
    std::vector<double> x;
    double v;
    while (std::fread(&v, sizeof v, 1, f) == 1) x.push_back(v);
    std::fclose(f);
    for (double &y : x) y = is_exp ? epdev::exp64(y) : epdev::log64(y);
    FILE *g = std::fopen(argv[3], "wb");
    if (!g || std::fwrite(x.data(), sizeof(double), x.size(), g) != x.size()) return 4;
    std::fclose(g);
    return 0;
}
