// Host build of the cell models' FP64 exponential: reads binary doubles from
// the file named by argv[1], writes exp64 of each to the file named by argv[2].
#include "cellmodels.hpp"
#include <cstdio>
#include <vector>

int main(int argc, char **argv) {
    if (argc != 3) return 2;
    FILE *f = std::fopen(argv[1], "rb");
    if (!f) return 3;
    std::vector<double> x;
    double v;
    while (std::fread(&v, sizeof v, 1, f) == 1) x.push_back(v);
    std::fclose(f);
    for (double &y : x) y = epdev::exp64(y);
    FILE *g = std::fopen(argv[2], "wb");
    if (!g || std::fwrite(x.data(), sizeof(double), x.size(), g) != x.size()) return 4;
    std::fclose(g);
    return 0;
}
