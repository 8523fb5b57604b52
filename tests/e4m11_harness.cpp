// Host harness for the e4m11 storage conversions of the HIP library
// (paper_2201_11330_amd/csrc/e4m11.hpp, compiled here as host code):
//   e4m11_harness encode <in.f32> <out.u16>   FP32 values -> codes
//   e4m11_harness decode <out.f32>            all 65536 codes -> FP32
#include <cstdio>
#include <string_view>
#include <vector>

#include "../paper_2201_11330_amd/csrc/e4m11.hpp"

int main(int argc, char** argv)
{
    using namespace imexlbm;
    if (argc == 4 && std::string_view(argv[1]) == "encode") {
        FILE* in = std::fopen(argv[2], "rb");
        if (!in) return 2;
        std::vector<float> v;
        float x;
        while (std::fread(&x, 4, 1, in) == 1) v.push_back(x);
        std::fclose(in);
        std::vector<uint16_t> out(v.size());
        for (size_t i = 0; i < v.size(); ++i) out[i] = e4m11_from_float(v[i]).bits;
        FILE* o = std::fopen(argv[3], "wb");
        if (!o) return 2;
        std::fwrite(out.data(), 2, out.size(), o);
        std::fclose(o);
        return 0;
    }
    if (argc == 3 && std::string_view(argv[1]) == "decode") {
        std::vector<float> out(65536);
        for (uint32_t c = 0; c < 65536; ++c) out[c] = e4m11_to_float(e4m11{uint16_t(c)});
        FILE* o = std::fopen(argv[2], "wb");
        if (!o) return 2;
        std::fwrite(out.data(), 4, out.size(), o);
        std::fclose(o);
        return 0;
    }
    std::fprintf(stderr, "usage: e4m11_harness encode <in.f32> <out.u16> | decode <out.f32>\n");
    return 1;
}
