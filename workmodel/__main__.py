from workmodel import main

main()
