// Empty stand-in for the HIP runtime header: the host checks compile device headers that need
// nothing from it beyond what they define themselves.
#pragma once
